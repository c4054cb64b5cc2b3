/*
 * fd.h -- batched forward dynamics of serial articulated chains on MI355X (gfx950).
 *
 * Method: Yang, Wu and Pan, "A Novel GPU-based Parallel Implementation Scheme
 * and Performance Analysis of Robot Forward Dynamics Algorithms" (arXiv
 * 1609.06779). Joint accelerations qdd are computed from joint torques tau,
 * positions q and velocities qd (Sec. II-C, eq. (eq-motion), (tau-bias)):
 *
 *     qdd = M(q)^-1 (tau - tau_bias(q, qd)),
 *
 * by one of three factorisations of M^-1: the joint space inertia inversion
 * algorithm (JSIIA, Sec. II-C), the articulated-body inertia algorithm (ABIA,
 * Sec. II-C) or the constraint force algorithm (CFA, Sec. III, Algorithm 1),
 * built from two solvers: a parallel scan for block bi-diagonal systems
 * (Sec. II-B) and odd-even elimination for block tri-diagonal systems
 * (Sec. IV, Algorithm 2). Both solvers are also exported on their own.
 *
 * Conventions. A robot is a serial chain of n revolute joints on a fixed base.
 * Twists are (w; v), wrenches (n; f). Link frame i sits on joint i's axis; its
 * pose in frame i-1 is T_{i-1,i}(q_i) = (Rhome_i Rot(axis_i, q_i), offset_i).
 * Branched robots (trees, beyond the paper's serial chains) name a parent per
 * link, and i-1 above reads that parent. The articulated-body algorithm takes
 * any numbering with parents before children (fd_forward with FD_ALGO_ABIA,
 * fd_forward_persistent, fd_backward). The lane-per-link paths (FD_ALGO_JSIIA,
 * fd_inverse, fd_joint_inertia) need the links of each robot numbered
 * depth-first, so that every subtree is a run of consecutive links. The CFA
 * (both forms) and FD_ALGO_ABIA_SCAN take serial chains only. A path that does not take the model returns
 * FD_ERR_UNSUPPORTED; FD_ALGO_AUTO picks one that does.
 * Gravity acts as a base acceleration (the "const." terms of eq. (EOM-full));
 * there is no force at the end effector. SI units, angles in radians.
 *
 * Layout. Per-link arrays of a batch are packed chain after chain: chain b
 * owns entries [start_b, start_b + n_b) of q, qd, tau, qdd. start_b is b * n
 * for batches whose chains all have n links (offsets == NULL), else offsets[b].
 *
 * Ownership and threading. The caller owns every state, output and workspace
 * buffer (device memory) and the stream; calls only enqueue work on that
 * stream, never allocate and never synchronise it (fd_init and fd_destroy
 * excepted). Buffers must stay valid until the stream has passed the call.
 * The model is read-only after fd_init, so calls on different streams may
 * overlap; a workspace must not be shared by calls that overlap.
 *
 * Errors. Argument checks are synchronous and return a status without
 * enqueueing anything. A launch failure returns FD_ERR_DEVICE. No C++
 * exception crosses this interface. Non-finite inputs give non-finite outputs.
 */
#ifndef FD_H
#define FD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FD_OK = 0,
    FD_ERR_INVALID_ARG = -1,   /* a null pointer, size or value out of range, inconsistent batch */
    FD_ERR_UNSUPPORTED = -2,   /* valid request this library does not handle (chain too long, ...) */
    FD_ERR_OUT_OF_MEMORY = -3, /* fd_init could not allocate device memory */
    FD_ERR_DEVICE = -4,        /* a HIP call or kernel launch failed */
    FD_ERR_WORKSPACE = -5      /* workspace missing or smaller than fd_workspace_size */
} fd_status_t;

/* FD_ALGO_ABIA runs one chain per lane (three serial sweeps; for large batches).
 * FD_ALGO_ABIA_SCAN is the same algorithm with a group of lanes per chain: the
 * serial articulated-inertia recursion spread over the 6x6 entries, then its
 * two bi-diagonal systems by the parallel scan (Sec. II-C, Sec. II-B); for
 * small batches (one robot: latency). FD_ALGO_CFA_PROJ is the constraint force
 * algorithm without a basis W of the constraint forces (Sec. III-B; Sec. VI
 * leaves the choice of W open): the projectors P_i = I - S_i S_i^T in its
 * place give a 6x6 block tri-diagonal system P Phi P + S S^T, solved by the
 * same odd-even elimination, whose solution is W F_c for every W. Both take
 * serial chains only. */
typedef enum {
    FD_ALGO_ABIA = 0,
    FD_ALGO_JSIIA = 1,
    FD_ALGO_CFA = 2,
    FD_ALGO_AUTO = 3,
    FD_ALGO_ABIA_SCAN = 4,
    FD_ALGO_CFA_PROJ = 5
} fd_algo_t;
typedef enum { FD_F64 = 0, FD_F32 = 1 } fd_dtype_t;

typedef struct fd_model fd_model_t; /* opaque, device resident, owned by the library */

/* Robot set, host pointers, FP64, copied by fd_init. Links of all robots are
 * packed robot after robot; robot r has n_links[r] >= 1 links. */
typedef struct {
    int32_t num_robots;
    const int32_t* n_links;  /* [num_robots] */
    const double* axis;      /* [L][3] joint axis in frame i (non-zero; normalised by fd_init) */
    const double* home_rot;  /* [L][9] row-major Rhome_i, or NULL for identity. Must be a rotation
                                to within 1e-6 (|R^T R - I| entrywise, det R); fd_init replaces it
                                by the nearest rotation (the orthogonal factor of its polar
                                decomposition), so every path reads one and the same rotation. */
    const double* offset;    /* [L][3] origin of frame i in frame i-1 */
    const double* mass;      /* [L] > 0 */
    const double* com;       /* [L][3] centre of mass in frame i */
    const double* inertia;   /* [L][6] SPD inertia about the COM, frame-i axes: xx yy zz xy xz yz */
    double gravity[3];       /* gravitational acceleration in the base frame, e.g. {0, 0, -9.81} */
    const int32_t* parent;   /* [L] parent of link i within its robot (0-based, < i), -1 = the base;
                                NULL: every robot is a serial chain (parent i-1). The pose, offset
                                and home rotation of link i are then taken in its parent's frame. */
} fd_model_desc_t;

/* A batch of chains (device pointers). */
typedef struct {
    int32_t batch;             /* number of chains, >= 0 */
    const int32_t* robot_id;   /* [batch] robot of chain b, or NULL: chain b uses robot b
                                  (every chain uses robot 0 when the model has one robot) */
    const int64_t* offsets;    /* [batch + 1] first entry of chain b, or NULL when all chains of
                                  the batch have the same length (start_b = b * n) */
    int32_t max_links;         /* 0, or an upper bound on the links of every chain of the batch:
                                  lane groups and workspaces are sized to the smaller of it and
                                  the longest robot the batch can name (with robot ids, the
                                  model's longest). A chain longer than the bound is not solved:
                                  its outputs are set to NaN. Must be 0..256. */
} fd_batch_t;

/* Upload a robot set in the given precision (FD_F32 rounds every parameter).
 * Validates masses, inertias, axes, rotations and parents; FD_ERR_INVALID_ARG if
 * any is out of range. Synchronous. On success *out owns device memory until fd_destroy. */
fd_status_t fd_init(const fd_model_desc_t* desc, fd_dtype_t dtype, fd_model_t** out);
void fd_destroy(fd_model_t* model);
fd_dtype_t fd_model_dtype(const fd_model_t* model);
/* Longest chain any algorithm of this library takes for the model's precision (JSIIA may be lower;
 * 0 for an algorithm that does not take the model's branched robots). */
int32_t fd_max_links(const fd_model_t* model, fd_algo_t algo);

/* Bytes of workspace fd_forward needs for this batch and algorithm (0 if none).
 * Reads no device memory: of robot_id and offsets only whether they are NULL
 * matters (the same holds for the other *_workspace_size calls). */
fd_status_t fd_workspace_size(const fd_model_t* model, const fd_batch_t* batch, fd_algo_t algo, size_t* bytes);

/* The algorithm FD_ALGO_AUTO takes for this batch (fd_set_auto_table), and
 * whether it runs as the persistent launch of fd_forward_persistent
 * (*persistent = 1; may be NULL). Like fd_workspace_size, it reads no device
 * memory: of robot_id and offsets only whether they are NULL matters. */
fd_status_t fd_auto_algo(const fd_model_t* model, const fd_batch_t* batch, fd_algo_t* algo, int* persistent);

/* Forward dynamics, eq. (tau-bias): qdd = M(q)^-1 (tau - tau_bias(q, qd)).
 * q, qd, tau, qdd: device arrays of the model's precision (double or float),
 * packed per chain. algo FD_ALGO_AUTO picks by the batch's longest chain and its
 * size (fd_set_auto_table); where that is ABIA on a batch with offsets, it runs
 * the persistent launch of fd_forward_persistent (grid 0), whose results are the
 * same bit for bit; fd_workspace_size with FD_ALGO_AUTO sizes the workspace for
 * the path AUTO takes. hip_stream: a hipStream_t (NULL = default stream).
 * Asynchronous. */
fd_status_t fd_forward(const fd_model_t* model, const fd_batch_t* batch, const void* q, const void* qd,
                       const void* tau, void* qdd, fd_algo_t algo, void* workspace, size_t ws_bytes,
                       void* hip_stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * computation as fd_forward (same kernels, same results bit for bit), with
 * the workspace taken from a scratch array of FD_NOALLOC_SCRATCH_BYTES that
 * the library holds on each GPU from its first fd_init on that GPU until the
 * process ends. No call allocates or frees memory. FD_ERR_WORKSPACE when the
 * batch needs more than FD_NOALLOC_SCRATCH_BYTES (fd_workspace_size with the
 * same arguments tells in advance); the algorithms without a workspace
 * (JSIIA, CFA) have no such limit. Every call on one GPU shares that GPU's
 * array, so calls that overlap on one GPU (concurrent streams, or threads)
 * race and give wrong results: serialise them. What must start at zero (the
 * persistent launch's tile counter and length histogram) is cleared by a
 * kernel inside each call, never by a memset. Asynchronous. */
#define FD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fd_status_t fd_forward_noalloc(const fd_model_t* model, const fd_batch_t* batch, const void* q, const void* qd,
                               const void* tau, void* qdd, fd_algo_t algo, void* hip_stream);

/* Forward dynamics of a batch, typically ragged, in one persistent launch of the
 * articulated-body algorithm (Sec. II-C). Small planning kernels first sort the
 * batch's chains on the device by decreasing length (into the workspace);
 * then `grid` resident wavefronts take 64-chain tiles of that order from an
 * atomic counter until none is left, so each tile holds chains of nearly
 * equal length and the longest go first. grid = 0 takes the default set by
 * fd_set_persistent_grid, or without one the number of wavefronts the GPU
 * holds at once; either way the launch takes at most one wavefront per
 * 64-chain tile of the batch. Results equal fd_forward(...,
 * FD_ALGO_ABIA, ...) bit for bit. The workspace must hold
 * fd_persistent_workspace_size bytes for the same batch and grid. Asynchronous. */
fd_status_t fd_persistent_workspace_size(const fd_model_t* model, const fd_batch_t* batch, int32_t grid,
                                         size_t* bytes);
fd_status_t fd_forward_persistent(const fd_model_t* model, const fd_batch_t* batch, const void* q, const void* qd,
                                  const void* tau, void* qdd, int32_t grid, void* workspace, size_t ws_bytes,
                                  void* hip_stream);

/* Reverse-mode derivative of fd_forward (a vector-Jacobian product). Given
 * qdd = FD(q, qd, tau) and a cotangent grad_qdd, writes
 *     grad_tau = lambda = M(q)^-1 grad_qdd,
 *     [grad_q; grad_qd] = -(d ID / d(q, qd))^T lambda   at (q, qd, qdd),
 * the implicit-function theorem applied to ID(q, qd, qdd) = tau (eq. (eq-motion)).
 * algo names the factorisation of M^-1 that gives lambda, as in fd_forward
 * (Sec. II-C, Sec. III): FD_ALGO_ABIA runs the articulated-body recursion inside
 * the reverse-mode kernel; FD_ALGO_JSIIA and FD_ALGO_CFA run their forward
 * kernel on M lambda = grad_qdd (tau_delta := grad_qdd: zero velocity, no
 * gravity); FD_ALGO_AUTO picks as fd_forward does. The transposed inverse
 * dynamics is one lane-per-chain kernel for every algo. qdd may be NULL: it is
 * then computed from (q, qd, tau) by the same algorithm first (tau is read only
 * then and may otherwise be NULL). accumulate != 0 adds to the three gradient
 * arrays instead of overwriting them. All arrays are device arrays of the
 * model's precision, packed per chain; the workspace must hold
 * fd_backward_workspace_size bytes for the same batch and algo. Asynchronous.
 * FD_ERR_UNSUPPORTED where fd_forward would refuse the algorithm. */
fd_status_t fd_backward_workspace_size(const fd_model_t* model, const fd_batch_t* batch, fd_algo_t algo,
                                       size_t* bytes);
fd_status_t fd_backward(const fd_model_t* model, const fd_batch_t* batch, const void* q, const void* qd,
                        const void* tau, const void* qdd, const void* grad_qdd, void* grad_q, void* grad_qd,
                        void* grad_tau, fd_algo_t algo, int accumulate, void* workspace, size_t ws_bytes,
                        void* hip_stream);

/* One semi-implicit Euler step of a rollout, elementwise over count entries:
 * qd_next = qd + dt qdd, q_next = q + dt qd_next. Outputs may alias inputs
 * entry by entry. Asynchronous. */
fd_status_t fd_euler_step(fd_dtype_t dtype, int64_t count, double dt, const void* q, const void* qd, const void* qdd,
                          void* q_next, void* qd_next, void* hip_stream);
/* Its adjoint: from the cotangents of (q_next, qd_next) writes those of q, qd
 * and qdd (overwriting): grad_qd = grad_qd_next + dt grad_q_next,
 * grad_q = grad_q_next, grad_qdd = dt grad_qd. Asynchronous. */
fd_status_t fd_euler_step_backward(fd_dtype_t dtype, int64_t count, double dt, const void* grad_q_next,
                                   const void* grad_qd_next, void* grad_q, void* grad_qd, void* grad_qdd,
                                   void* hip_stream);

/* Inverse dynamics, eq. (EOM-full) (CalcInvDyn of Algorithm 1):
 * tau = M(q) qdd + tau_bias(q, qd), with gravity when `gravity` != 0.
 * qdd may be NULL (zero: tau is then the bias torque). Asynchronous. */
fd_status_t fd_inverse(const fd_model_t* model, const fd_batch_t* batch, const void* q, const void* qd,
                       const void* qdd, int gravity, void* tau, void* hip_stream);

/* Joint-space inertia M(q) = S^T (I - Gamma)^-T J (I - Gamma)^-1 S (Sec. II-C) as
 * the JSIIA builds it. Uniform batches only (offsets NULL): chain b's n x n
 * row-major block starts at m_out + b * n * n. Asynchronous. */
fd_status_t fd_joint_inertia(const fd_model_t* model, const fd_batch_t* batch, const void* q, void* m_out,
                             void* hip_stream);

/* Segmented scan for block bi-diagonal systems (Sec. II-B):
 *     x_i = B_i x_{i-1} + c_i within each segment (x before the segment = 0),
 * or with reverse != 0, x_i = B_i x_{i+1} + c_i. b: [N][6][6] row-major,
 * c, x: [N][6], device; offsets: device [segments + 1]; every segment at most
 * 256 long. dtype selects double or float. Asynchronous. */
fd_status_t fd_scan6(fd_dtype_t dtype, int32_t segments, const int64_t* offsets, int32_t max_len, const void* b,
                     const void* c, int reverse, void* x, void* hip_stream);

/* Odd-even elimination (Sec. IV, Algorithm 2) for symmetric positive definite
 * block tri-diagonal systems with 6x6 blocks, eq. (A_mat): system s has rows
 * offsets[s] .. offsets[s+1]-1 with diagonal blocks d[i] and upper blocks u[i]
 * coupling rows i and i+1 (u of a system's last row is ignored); solves
 * A x = r. d, u: [N][6][6] row-major, r, x: [N][6]; at most 256 rows per
 * system. status (device int, may be NULL) gets bit 0 set when a pivot was
 * not positive (A not SPD) and bit 1 when a system is longer than max_len (left
 * untouched). Asynchronous. */
fd_status_t fd_btd_solve6(fd_dtype_t dtype, int32_t segments, const int64_t* offsets, int32_t max_len,
                          const void* d, const void* u, const void* r, void* x, int* status, void* hip_stream);

/* Choice table for FD_ALGO_AUTO, per precision: table[n * 21 + k] (n = 1..256,
 * k = 0..20) is the algorithm (any but FD_ALGO_AUTO) for batches whose
 * longest chain has n links and whose size rounds to 2^k chains; produced by
 * the autotuner from measured launch times. Host pointer, 257 * 21 bytes,
 * copied. NULL restores the built-in choice. Not safe to call while another
 * thread is inside fd_forward. FD_ERR_INVALID_ARG for a bad dtype or entry. */
fd_status_t fd_set_auto_table(fd_dtype_t dtype, const int8_t* table);

/* Default grid of persistent launches (fd_forward_persistent with grid 0, and
 * the persistent launch AUTO takes), per precision; produced by the autotuner.
 * 0 restores the resident capacity. Not safe to call while another thread is
 * inside fd_forward. FD_ERR_INVALID_ARG for a bad dtype or a negative grid. */
fd_status_t fd_set_persistent_grid(fd_dtype_t dtype, int32_t grid);

const char* fd_status_string(fd_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* FD_H */
