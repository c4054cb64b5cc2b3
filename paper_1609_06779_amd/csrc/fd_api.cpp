// fd_api.cpp -- host runtime of the C-ABI (include/fd.h): argument checks,
// model upload, tile choice and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/fd.h"
#include "kernels.h"

// Scratch memory of fd_forward_noalloc: one copy per GPU, held from the
// library's load until the process ends. In host code `scratch` names a
// host-side stand-in, never the device copy: host code only ever uses the
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[FD_NOALLOC_SCRATCH_BYTES];

struct fd_model {
    fd_dtype_t dtype = FD_F64;
    int32_t num_robots = 0;
    int64_t total_links = 0;
    std::vector<int32_t> n_links;     // host copy
    std::vector<int32_t> prefix_max;  // max n over robots 0..r
    std::vector<uint8_t> prefix_uni;  // robots 0..r all have n_links[0] links
    int32_t nmax = 0;
    bool uniform = false;
    double g[3] = {0, 0, 0};
    void* d_fields = nullptr;         // T[MF_COUNT][total_links]
    void* d_il = nullptr;             // T[IL_COUNT][nmax][num_robots], columns by decreasing length
    int64_t* d_link_start = nullptr;
    int32_t* d_n_links = nullptr;
    int32_t* d_slot = nullptr;        // [num_robots] column of each robot in d_il
    int32_t* d_slot_robot = nullptr;  // [num_robots] robot of each column
    bool tree = false;                // some robot is branched (a link's parent is not link i-1)
    bool depth_first = true;          // every robot's links are numbered depth-first (subtrees are runs)
    bool shared_topology = true;      // robots of one length share one parent array
    int32_t* d_tree = nullptr;        // [nmax][num_robots] tree codes (see lanes.h), null without branches
};

namespace {

constexpr int kMaxLinks = 256;

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

bool valid_rotation(const double* r) {
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(r[k])) return false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double d = r[3 * i] * r[3 * j] + r[3 * i + 1] * r[3 * j + 1] + r[3 * i + 2] * r[3 * j + 2];
            if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-6) return false;
        }
    double det = r[0] * (r[4] * r[8] - r[5] * r[7]) - r[1] * (r[3] * r[8] - r[5] * r[6]) +
                 r[2] * (r[3] * r[7] - r[4] * r[6]);
    return std::fabs(det - 1.0) < 1e-6;
}

// The rotation nearest to r in the Frobenius norm (the orthogonal factor of
// its polar decomposition), for an r that valid_rotation accepted: Newton-Schulz
// steps X <- X (3 I - X^T X) / 2 converge quadratically from ||X^T X - I|| <= 1e-6,
// so two steps reach rounding level; a few more cost nothing.
void polar_rotation(const double* r, double* out) {
    double x[9];
    std::memcpy(x, r, sizeof(x));
    for (int it = 0; it < 4; ++it) {
        double g[9], y[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                g[3 * i + j] = (i == j ? 3.0 : 0.0) -
                               (x[i] * x[j] + x[3 + i] * x[3 + j] + x[6 + i] * x[6 + j]);   // 3 I - X^T X
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                y[3 * i + j] = 0.5 * (x[3 * i] * g[j] + x[3 * i + 1] * g[3 + j] + x[3 * i + 2] * g[6 + j]);
        std::memcpy(x, y, sizeof(x));
    }
    std::memcpy(out, x, sizeof(x));
}

bool valid_inertia(const double* in) {
    for (int k = 0; k < 6; ++k)
        if (!std::isfinite(in[k])) return false;
    double a00 = in[0], a11 = in[1], a22 = in[2], a01 = in[3], a02 = in[4], a12 = in[5];
    double m2 = a00 * a11 - a01 * a01;
    double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
    return a00 > 0 && m2 > 0 && det > 0;
}

int pow2_lanes(int n) {
    int p = 8;
    while (p < n) p <<= 1;
    return p;
}

template <typename T> fdk::ModelView<T> view(const fd_model* m) {
    fdk::ModelView<T> v;
    v.base = static_cast<const T*>(m->d_fields);
    v.stride = m->total_links;
    v.link_start = m->d_link_start;
    v.n_links = m->d_n_links;
    v.num_robots = m->num_robots;
    for (int k = 0; k < 3; ++k) v.g[k] = (T)m->g[k];
    v.il = static_cast<const T*>(m->d_il);
    v.il_fstride = (int64_t)m->nmax * m->num_robots;
    v.slot = m->d_slot;
    v.tree = m->d_tree;
    return v;
}

struct BatchPlan {
    fdk::ChainMap cm;
    int nmax;
};

fd_status_t plan_batch(const fd_model* m, const fd_batch_t* b, BatchPlan* p) {
    if (!m || !b || b->batch < 0 || b->max_links < 0 || b->max_links > kMaxLinks) return FD_ERR_INVALID_ARG;
    p->cm.robot_id = b->robot_id;
    p->cm.offsets = b->offsets;
    p->cm.batch = b->batch;
    p->cm.n_uniform = 0;
    p->cm.n_cap = 0;
    p->nmax = 0;
    if (b->batch == 0) return FD_OK;
    bool uni;
    int n0;
    if (b->robot_id == nullptr) {
        if (m->num_robots == 1) {
            p->nmax = m->n_links[0];
            uni = true;
        } else {
            if (b->batch > m->num_robots) return FD_ERR_INVALID_ARG;
            p->nmax = m->prefix_max[b->batch - 1];
            uni = m->prefix_uni[b->batch - 1] != 0;
        }
        n0 = m->n_links[0];
    } else {
        p->nmax = m->nmax;
        uni = m->uniform;
        n0 = m->n_links[0];
    }
    if (b->offsets == nullptr) {
        if (!uni) return FD_ERR_INVALID_ARG;
        p->cm.n_uniform = n0;
    }
    if (b->max_links > 0) p->nmax = std::min(p->nmax, b->max_links);
    p->cm.n_cap = p->nmax;
    return FD_OK;
}

// Bytes of interleaved model and workspace that a lane-per-chain launch
// streams per sweep. Past the last-level cache (256 MB Infinity Cache on
// MI355X) nothing survives until the next sweep, so the kernels stream them
// with non-temporal accesses and leave the cache to the chain state.
constexpr size_t kLastLevelCache = size_t(256) << 20;
bool stream_model(const fd_model* m, int batch, int nmax) {
    const size_t esz = m->dtype == FD_F64 ? sizeof(double) : sizeof(float);
    return (size_t)batch * nmax * (fdk::IL_COUNT + 7) * esz > kLastLevelCache;
}

fd_status_t from_hip(hipError_t e) {
    if (e == hipSuccess) return FD_OK;
    if (e == hipErrorInvalidConfiguration) return FD_ERR_UNSUPPORTED;
    return FD_ERR_DEVICE;
}

// AUTO choice tables (per precision), [n][log2 batch]; empty = built-in rule.
std::vector<int8_t> g_auto[2];

int log2_bucket(int batch) {
    int k = 0;
    while (k < 20 && (1 << (k + 1)) <= batch) ++k;
    // round to nearest power of two
    if (k < 20 && batch - (1 << k) > (1 << (k + 1)) - batch) ++k;
    return k;
}

fd_algo_t pick_algo(const fd_model* m, int nmax, int batch) {
    const std::vector<int8_t>& t = g_auto[m->dtype == FD_F64 ? 0 : 1];
    // built-in rule: one lane per chain wins once the batch fills the GPU
    fd_algo_t a = FD_ALGO_ABIA;
    if (!t.empty() && nmax >= 1 && nmax <= kMaxLinks) a = (fd_algo_t)t[nmax * 21 + log2_bucket(batch)];
    // branched robots: the CFA is built for serial chains, JSIIA for depth-first numbering
    if (m->tree && (a == FD_ALGO_CFA || a == FD_ALGO_CFA_PROJ || a == FD_ALGO_ABIA_SCAN ||
                    (a == FD_ALGO_JSIIA && !m->depth_first)))
        a = FD_ALGO_ABIA;
    // Robots of different topologies in one wavefront make the lane-per-chain
    // ABIA diverge at every branch point of any of its lanes (65536 trees of 64
    // links: 2.1 ms, against 0.66 ms with one shared topology); JSIIA puts one
    // tree on a lane group and does not diverge (1.1 ms either way).
    const int jmax = m->dtype == FD_F64 ? fdk::jsiia_max_np<double>() : fdk::jsiia_max_np<float>();
    if (m->tree && !m->shared_topology && m->depth_first && a == FD_ALGO_ABIA && pow2_lanes(nmax) <= jmax)
        a = FD_ALGO_JSIIA;
    return a;
}

// AUTO on a ragged batch (offsets given) that picks ABIA runs the persistent,
// length-sorted launch: the same results bit for bit, without every wavefront
// running to the longest chain of its 64.
bool auto_persistent(const fd_batch_t* b, fd_algo_t picked) { return b->offsets != nullptr && picked == FD_ALGO_ABIA; }

// Lane groups of a lane-per-link launch, or FD_ERR_UNSUPPORTED when the
// algorithm does not take this model or chain length.
template <typename T> fd_status_t lane_path_check(const fd_model* m, fd_algo_t algo, int np) {
    if (algo == FD_ALGO_JSIIA && ((m->tree && !m->depth_first) || np > fdk::jsiia_max_np<T>())) return FD_ERR_UNSUPPORTED;
    if ((algo == FD_ALGO_CFA || algo == FD_ALGO_CFA_PROJ || algo == FD_ALGO_ABIA_SCAN) && m->tree)
        return FD_ERR_UNSUPPORTED;
    return FD_OK;
}

template <typename T>
fd_status_t forward_t(const fd_model* m, const BatchPlan& p, const void* q, const void* qd, const void* tau,
                      void* qdd, fd_algo_t algo, void* ws, size_t ws_bytes, hipStream_t st,
                      const fdk::FdOut<T>& o = fdk::FdOut<T>{}) {
    const auto v = view<T>(m);
    const T* tq = static_cast<const T*>(q);
    const T* tqd = static_cast<const T*>(qd);
    const T* tt = static_cast<const T*>(tau);
    T* out = static_cast<T*>(qdd);
    const int np = pow2_lanes(p.nmax);
    const fd_status_t ok = lane_path_check<T>(m, algo, np);
    if (ok != FD_OK) return ok;
    if (!out && !o.aux) return FD_ERR_INVALID_ARG;   // the kernels need somewhere to put qdd
    switch (algo) {
        case FD_ALGO_ABIA: {
            size_t need = fdk::abia_workspace_elems(p.cm.batch, p.nmax, m->tree) * sizeof(T);
            if (!ws || ws_bytes < need) return FD_ERR_WORKSPACE;
            return from_hip(fdk::launch_abia<T>(v, p.cm, p.nmax, tq, tqd, tt, out, static_cast<T*>(ws),
                                                stream_model(m, p.cm.batch, p.nmax), o, st));
        }
        case FD_ALGO_JSIIA:
            return from_hip(fdk::launch_jsiia<T>(np, v, p.cm, tq, tqd, tt, out, nullptr, o, st));
        case FD_ALGO_CFA:
        case FD_ALGO_CFA_PROJ:
            return from_hip(fdk::launch_cfa<T>(np, v, p.cm, tq, tqd, tt, out, nullptr, o, algo == FD_ALGO_CFA_PROJ, st));
        case FD_ALGO_ABIA_SCAN:
            return from_hip(fdk::launch_abia_scan<T>(np, v, p.cm, tq, tqd, tt, out, o, st));
        default:
            return FD_ERR_INVALID_ARG;
    }
}

// Reverse mode. The VJP kernel's workspace comes first; an ABIA forward that
// recomputes qdd (qdd == NULL) takes its own workspace after it.
template <typename T>
size_t backward_bytes(const fd_model* m, const BatchPlan& p, fd_algo_t algo) {
    const size_t vjp = fdk::vjp_workspace_elems(p.cm.batch, p.nmax, m->tree) * sizeof(T);
    const size_t fwd = algo == FD_ALGO_ABIA ? fdk::abia_workspace_elems(p.cm.batch, p.nmax, m->tree) * sizeof(T) : 0;
    return vjp + fwd;
}

template <typename T>
fd_status_t backward_t(const fd_model* m, const BatchPlan& p, const void* q, const void* qd, const void* tau,
                       const void* qdd, const void* gqdd, void* gq, void* gqd, void* gtau, fd_algo_t algo,
                       int accumulate, void* ws, size_t ws_bytes, hipStream_t st) {
    const int np = pow2_lanes(p.nmax);
    fd_status_t s = lane_path_check<T>(m, algo, np);
    if (s != FD_OK) return s;
    if (!ws || ws_bytes < backward_bytes<T>(m, p, algo)) return FD_ERR_WORKSPACE;
    T* vws = static_cast<T*>(ws);
    const size_t vjp_elems = fdk::vjp_workspace_elems(p.cm.batch, p.nmax, m->tree);
    fdk::FdOut<T> to_ws;                          // a result handed to the VJP kernel through its workspace
    to_ws.aux = vws;
    to_ws.aux_nmax = p.nmax;
    to_ws.aux_fields = fdk::vjp_fields_of(m->tree);
    if (!qdd) {                                   // qdd = FD(q, qd, tau) by the same factorisation
        to_ws.aux_field = fdk::vjp_field_qdd();
        s = forward_t<T>(m, p, q, qd, tau, nullptr, algo, vws + vjp_elems, ws_bytes - vjp_elems * sizeof(T), st,
                         to_ws);
        if (s != FD_OK) return s;
    }
    const bool lam_in = algo != FD_ALGO_ABIA;
    if (lam_in) {                                 // lambda = M^-1 g by the JSIIA or the CFA, into grad_tau and the workspace
        fdk::FdOut<T> lam = to_ws;
        lam.aux_field = fdk::vjp_field_lambda();
        lam.solve = 1;
        lam.accumulate = accumulate;
        s = forward_t<T>(m, p, q, nullptr, gqdd, gtau, algo, nullptr, 0, st, lam);
        if (s != FD_OK) return s;
    }
    return from_hip(fdk::launch_fd_vjp<T>(view<T>(m), p.cm, p.nmax, static_cast<const T*>(q),
                                          static_cast<const T*>(qd), static_cast<const T*>(qdd),
                                          static_cast<const T*>(gqdd), static_cast<T*>(gq), static_cast<T*>(gqd),
                                          static_cast<T*>(gtau), accumulate, lam_in, vws,
                                          stream_model(m, p.cm.batch, p.nmax), st));
}

// The device address of the current GPU's copy of `scratch`, looked up once
// per device (with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

fd_status_t scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FD_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FD_ERR_DEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FD_OK;
}

}  // namespace

extern "C" {

fd_status_t fd_init(const fd_model_desc_t* d, fd_dtype_t dtype, fd_model_t** out) {
    if (!d || !out || d->num_robots < 1 || !d->n_links || !d->axis || !d->offset || !d->mass || !d->com ||
        !d->inertia || (dtype != FD_F64 && dtype != FD_F32))
        return FD_ERR_INVALID_ARG;
    *out = nullptr;
    if (!finite3(d->gravity)) return FD_ERR_INVALID_ARG;
    int64_t total = 0;
    for (int r = 0; r < d->num_robots; ++r) {
        if (d->n_links[r] < 1 || d->n_links[r] > kMaxLinks) return FD_ERR_INVALID_ARG;
        total += d->n_links[r];
    }
    static const double kEye[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::vector<double> raw;
    std::vector<int64_t> parent_link;
    std::vector<int32_t> code;
    try {
        raw.resize((size_t)total * 25);
        parent_link.resize((size_t)total);
        code.assign((size_t)total, 0);
    } catch (const std::bad_alloc&) {
        return FD_ERR_OUT_OF_MEMORY;
    }
    // topology: parent links and the tree codes (lanes.h)
    bool tree = false, depth_first = true, shared_topology = true;
    std::map<int, int64_t> first_of_length;   // length -> start of the first robot of that length
    for (int64_t r = 0, s0 = 0; r < d->num_robots; s0 += d->n_links[r], ++r) {
        const int n = d->n_links[r];
        std::vector<int> par(n), size(n, 1);
        for (int i = 0; i < n; ++i) {
            const int p = d->parent ? d->parent[s0 + i] : i - 1;
            if (p < -1 || p >= i) return FD_ERR_INVALID_ARG;
            par[i] = p;
            parent_link[s0 + i] = p >= 0 ? s0 + p : -1;
            tree = tree || p != i - 1;
            // depth-first numbering: the parent of i is i - 1 or one of its ancestors
            int k = i - 1;
            while (k >= 0 && k != p) k = par[k];
            depth_first = depth_first && k == p;
        }
        const auto seen = first_of_length.emplace(n, s0);
        if (!seen.second && d->parent) {
            const int64_t f0 = seen.first->second;
            for (int i = 0; i < n && shared_topology; ++i) shared_topology = d->parent[f0 + i] == d->parent[s0 + i];
        }
        for (int i = n - 1; i >= 1; --i)
            if (par[i] >= 0) size[par[i]] += size[i];
        std::vector<uint8_t> reached(n, 0);
        for (int i = n - 1; i >= 0; --i) {   // children before parents, as in the backward sweep
            const int p = par[i];
            code[s0 + i] |= (p + 1) | ((i + size[i]) << 9) | (p >= 0 && p == i - 1 ? fdk::TREE_CHAIN : 0);
            if (p < 0 || p == i - 1) continue;
            code[s0 + p] |= fdk::TREE_BRANCH;
            if (!reached[p]) code[s0 + i] |= fdk::TREE_FIRST;
            reached[p] = 1;
        }
    }
    int64_t l = 0;
    for (int r = 0; r < d->num_robots; ++r) {
        for (int i = 0; i < d->n_links[r]; ++i, ++l) {
            const double* ax = d->axis + 3 * l;
            const double* hr = d->home_rot ? d->home_rot + 9 * l : kEye;
            if (!finite3(ax) || std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]) < 1e-12) return FD_ERR_INVALID_ARG;
            if (!valid_rotation(hr) || !finite3(d->offset + 3 * l) || !finite3(d->com + 3 * l)) return FD_ERR_INVALID_ARG;
            if (!std::isfinite(d->mass[l]) || !(d->mass[l] > 0)) return FD_ERR_INVALID_ARG;
            if (!valid_inertia(d->inertia + 6 * l)) return FD_ERR_INVALID_ARG;
            double* w = raw.data() + 25 * l;
            std::memcpy(w + 0, ax, 3 * sizeof(double));
            // every path (matrix, quaternion) then reads one and the same rotation
            polar_rotation(hr, w + 3);
            std::memcpy(w + 12, d->offset + 3 * l, 3 * sizeof(double));
            w[15] = d->mass[l];
            std::memcpy(w + 16, d->com + 3 * l, 3 * sizeof(double));
            std::memcpy(w + 19, d->inertia + 6 * l, 6 * sizeof(double));
        }
    }
    fd_model* m = new (std::nothrow) fd_model;
    if (!m) return FD_ERR_OUT_OF_MEMORY;
    m->dtype = dtype;
    m->num_robots = d->num_robots;
    m->total_links = total;
    m->n_links.assign(d->n_links, d->n_links + d->num_robots);
    m->prefix_max.resize(d->num_robots);
    m->prefix_uni.resize(d->num_robots);
    int32_t mx = 0;
    bool uni = true;
    for (int r = 0; r < d->num_robots; ++r) {
        mx = std::max(mx, d->n_links[r]);
        uni = uni && d->n_links[r] == d->n_links[0];
        m->prefix_max[r] = mx;
        m->prefix_uni[r] = uni;
    }
    m->nmax = mx;
    m->uniform = uni;
    m->tree = tree;
    m->depth_first = depth_first;
    m->shared_topology = shared_topology;
    for (int k = 0; k < 3; ++k) m->g[k] = d->gravity[k];
    // interleaved columns: robots by decreasing length, ties in robot order, so a
    // model of equal lengths keeps its order and 64 consecutive columns hold
    // robots of nearly equal length
    std::vector<int32_t> slot_robot(d->num_robots), slot(d->num_robots);
    for (int r = 0; r < d->num_robots; ++r) slot_robot[r] = r;
    std::stable_sort(slot_robot.begin(), slot_robot.end(),
                     [&](int32_t a, int32_t b) { return d->n_links[a] > d->n_links[b]; });
    for (int c = 0; c < d->num_robots; ++c) slot[slot_robot[c]] = c;
    std::vector<int64_t> starts(d->num_robots);
    std::vector<int32_t> column_of(total), index_of(total);
    int64_t s = 0;
    for (int r = 0; r < d->num_robots; ++r) {
        starts[r] = s;
        for (int i = 0; i < d->n_links[r]; ++i) {
            column_of[s + i] = slot[r];
            index_of[s + i] = i;
        }
        s += d->n_links[r];
    }
    const int64_t il_elems = (int64_t)fdk::IL_COUNT * mx * d->num_robots;
    std::vector<int32_t> tree_il;
    if (tree) {
        tree_il.assign((size_t)mx * d->num_robots, 0);
        for (int r = 0; r < d->num_robots; ++r)
            for (int i = 0; i < d->n_links[r]; ++i) tree_il[(size_t)i * d->num_robots + slot[r]] = code[starts[r] + i];
    }
    int32_t* d_ri = nullptr;
    const size_t esz = dtype == FD_F64 ? sizeof(double) : sizeof(float);
    double* d_raw = nullptr;
    int64_t* d_parent = nullptr;
    fd_status_t st = FD_OK;
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&m->d_fields, esz * fdk::MF_COUNT * total)) != hipSuccess ||
        (e = hipMalloc(&m->d_link_start, sizeof(int64_t) * d->num_robots)) != hipSuccess ||
        (e = hipMalloc(&m->d_n_links, sizeof(int32_t) * d->num_robots)) != hipSuccess ||
        (e = hipMalloc(&m->d_slot, sizeof(int32_t) * d->num_robots)) != hipSuccess ||
        (e = hipMalloc(&m->d_slot_robot, sizeof(int32_t) * d->num_robots)) != hipSuccess ||
        (e = hipMalloc(&d_raw, raw.size() * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&d_parent, sizeof(int64_t) * total)) != hipSuccess ||
        (tree && (e = hipMalloc(&m->d_tree, sizeof(int32_t) * tree_il.size())) != hipSuccess) ||
        (e = hipMalloc(&m->d_il, esz * il_elems)) != hipSuccess ||
        (e = hipMalloc(&d_ri, sizeof(int32_t) * 2 * total)) != hipSuccess) {
        st = e == hipErrorOutOfMemory ? FD_ERR_OUT_OF_MEMORY : FD_ERR_DEVICE;
    }
    if (st == FD_OK) {
        if (hipMemcpy(m->d_link_start, starts.data(), sizeof(int64_t) * starts.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(m->d_n_links, d->n_links, sizeof(int32_t) * d->num_robots, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(m->d_slot, slot.data(), sizeof(int32_t) * d->num_robots, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(m->d_slot_robot, slot_robot.data(), sizeof(int32_t) * d->num_robots, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(d_raw, raw.data(), raw.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_parent, parent_link.data(), sizeof(int64_t) * total, hipMemcpyHostToDevice) != hipSuccess ||
            (tree && hipMemcpy(m->d_tree, tree_il.data(), sizeof(int32_t) * tree_il.size(), hipMemcpyHostToDevice) !=
                         hipSuccess) ||
            hipMemcpy(d_ri, column_of.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_ri + total, index_of.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(m->d_il, 0, esz * il_elems) != hipSuccess ||
            fdk::launch_model_init(total, d_raw, d_parent, m->d_fields, dtype == FD_F32, nullptr) != hipSuccess ||
            fdk::launch_model_interleave(total, d_ri, d_ri + total, d->num_robots, (int64_t)mx * d->num_robots,
                                         m->d_fields, m->d_il, dtype == FD_F32, nullptr) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            st = FD_ERR_DEVICE;
    }
    if (d_raw) (void)hipFree(d_raw);
    if (d_parent) (void)hipFree(d_parent);
    if (d_ri) (void)hipFree(d_ri);
    void* scratch_ptr = nullptr;             // set-up of fd_forward_noalloc on this device
    if (st == FD_OK) st = scratch_address(&scratch_ptr);
    if (st != FD_OK) {
        fd_destroy(m);
        return st;
    }
    *out = m;
    return FD_OK;
}

void fd_destroy(fd_model_t* m) {
    if (!m) return;
    if (m->d_fields) (void)hipFree(m->d_fields);
    if (m->d_il) (void)hipFree(m->d_il);
    if (m->d_link_start) (void)hipFree(m->d_link_start);
    if (m->d_n_links) (void)hipFree(m->d_n_links);
    if (m->d_slot) (void)hipFree(m->d_slot);
    if (m->d_slot_robot) (void)hipFree(m->d_slot_robot);
    if (m->d_tree) (void)hipFree(m->d_tree);
    delete m;
}

fd_dtype_t fd_model_dtype(const fd_model_t* m) { return m ? m->dtype : FD_F64; }

int32_t fd_max_links(const fd_model_t* m, fd_algo_t algo) {
    if (!m) return 0;
    if (m->tree && (algo == FD_ALGO_CFA || algo == FD_ALGO_CFA_PROJ || algo == FD_ALGO_ABIA_SCAN ||
                    (algo == FD_ALGO_JSIIA && !m->depth_first)))
        return 0;
    if (algo == FD_ALGO_JSIIA) return m->dtype == FD_F64 ? fdk::jsiia_max_np<double>() : fdk::jsiia_max_np<float>();
    return kMaxLinks;
}

fd_status_t fd_workspace_size(const fd_model_t* m, const fd_batch_t* b, fd_algo_t algo, size_t* bytes) {
    if (!bytes) return FD_ERR_INVALID_ARG;
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (algo == FD_ALGO_AUTO) {
        algo = pick_algo(m, p.nmax, b->batch);
        if (auto_persistent(b, algo)) return fd_persistent_workspace_size(m, b, 0, bytes);
    }
    const size_t esz = m->dtype == FD_F64 ? sizeof(double) : sizeof(float);
    *bytes = algo == FD_ALGO_ABIA ? fdk::abia_workspace_elems(b->batch, p.nmax, m->tree) * esz : 0;
    return FD_OK;
}

fd_status_t fd_auto_algo(const fd_model_t* m, const fd_batch_t* b, fd_algo_t* algo, int* persistent) {
    if (!algo) return FD_ERR_INVALID_ARG;
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    *algo = pick_algo(m, p.nmax, b->batch);
    if (persistent) *persistent = auto_persistent(b, *algo) ? 1 : 0;
    return FD_OK;
}

fd_status_t fd_forward(const fd_model_t* m, const fd_batch_t* b, const void* q, const void* qd, const void* tau,
                       void* qdd, fd_algo_t algo, void* ws, size_t ws_bytes, void* hip_stream) {
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (algo < FD_ALGO_ABIA || algo > FD_ALGO_CFA_PROJ) return FD_ERR_INVALID_ARG;
    if (b->batch == 0) return FD_OK;
    if (!q || !qd || !tau || !qdd) return FD_ERR_INVALID_ARG;
    if (algo == FD_ALGO_AUTO) {
        algo = pick_algo(m, p.nmax, b->batch);
        if (auto_persistent(b, algo)) return fd_forward_persistent(m, b, q, qd, tau, qdd, 0, ws, ws_bytes, hip_stream);
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (m->dtype == FD_F64) return forward_t<double>(m, p, q, qd, tau, qdd, algo, ws, ws_bytes, st);
    return forward_t<float>(m, p, q, qd, tau, qdd, algo, ws, ws_bytes, st);
}

fd_status_t fd_forward_noalloc(const fd_model_t* m, const fd_batch_t* b, const void* q, const void* qd,
                               const void* tau, void* qdd, fd_algo_t algo, void* hip_stream) {
    size_t need = 0;
    fd_status_t s = fd_workspace_size(m, b, algo, &need);
    if (s != FD_OK) return s;
    if (need > FD_NOALLOC_SCRATCH_BYTES) return FD_ERR_WORKSPACE;
    void* ws = nullptr;
    if (need > 0 && (s = scratch_address(&ws)) != FD_OK) return s;
    return fd_forward(m, b, q, qd, tau, qdd, algo, ws, need > 0 ? FD_NOALLOC_SCRATCH_BYTES : 0, hip_stream);
}

// Default grid of persistent launches per precision (fd_set_persistent_grid; 0:
// the resident capacity).
int32_t g_persistent_grid[2] = {0, 0};

// Wavefronts of a persistent launch: the caller's grid, else (grid 0) the
// default set for the precision, else as many as the GPU holds at once; never
// more than the batch has 64-chain tiles, since a wavefront without a tile only
// exits (and each one holds workspace).
int persistent_grid(fd_dtype_t dtype, int32_t grid, int32_t batch) {
    int g = grid > 0 ? grid : g_persistent_grid[dtype == FD_F64 ? 0 : 1];
    if (g <= 0) {
        int dev = 0, cus = 256;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // one 64-thread workgroup per SIMD per wave slot the kernel's registers allow
        const int per_cu = dtype == FD_F64 ? 4 : 12;
        g = cus * per_cu;
    }
    const int tiles = (std::max(batch, 1) + 63) / 64;
    return std::min(g, tiles);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

fd_status_t fd_persistent_workspace_size(const fd_model_t* m, const fd_batch_t* b, int32_t grid, size_t* bytes) {
    if (!bytes || grid < 0) return FD_ERR_INVALID_ARG;
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    const size_t esz = m->dtype == FD_F64 ? sizeof(double) : sizeof(float);
    const int g = persistent_grid(m->dtype, grid, b->batch);
    *bytes = align256(fdk::persistent_plan_bytes(b->batch)) + fdk::abia_persistent_workspace_elems(g, p.nmax, m->tree) * esz;
    return FD_OK;
}

fd_status_t fd_forward_persistent(const fd_model_t* m, const fd_batch_t* b, const void* q, const void* qd,
                                  const void* tau, void* qdd, int32_t grid, void* ws, size_t ws_bytes,
                                  void* hip_stream) {
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (grid < 0) return FD_ERR_INVALID_ARG;
    if (b->batch == 0) return FD_OK;
    if (!q || !qd || !tau || !qdd) return FD_ERR_INVALID_ARG;
    const size_t esz = m->dtype == FD_F64 ? sizeof(double) : sizeof(float);
    const int g = persistent_grid(m->dtype, grid, b->batch);
    const size_t plan = align256(fdk::persistent_plan_bytes(b->batch));
    if (!ws || ws_bytes < plan + fdk::abia_persistent_workspace_elems(g, p.nmax, m->tree) * esz)
        return FD_ERR_WORKSPACE;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int32_t* planp = static_cast<int32_t*>(ws);
    void* abws = static_cast<char*>(ws) + plan;
    if (m->dtype == FD_F64)
        return from_hip(fdk::launch_abia_persistent<double>(view<double>(m), p.cm, p.nmax, g, (const double*)q,
                                                            (const double*)qd, (const double*)tau, (double*)qdd,
                                                            (double*)abws, planp, m->d_slot_robot,
                                                            stream_model(m, b->batch, p.nmax), st));
    return from_hip(fdk::launch_abia_persistent<float>(view<float>(m), p.cm, p.nmax, g, (const float*)q,
                                                       (const float*)qd, (const float*)tau, (float*)qdd, (float*)abws,
                                                       planp, m->d_slot_robot, stream_model(m, b->batch, p.nmax), st));
}

// The algorithm a reverse-mode call runs: AUTO takes fd_forward's choice.
fd_algo_t backward_algo(const fd_model* m, const BatchPlan& p, int batch, fd_algo_t algo) {
    return algo == FD_ALGO_AUTO ? pick_algo(m, p.nmax, batch) : algo;
}

fd_status_t fd_backward_workspace_size(const fd_model_t* m, const fd_batch_t* b, fd_algo_t algo, size_t* bytes) {
    if (!bytes) return FD_ERR_INVALID_ARG;
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (algo < FD_ALGO_ABIA || algo > FD_ALGO_CFA_PROJ) return FD_ERR_INVALID_ARG;
    algo = backward_algo(m, p, b->batch, algo);
    *bytes = m->dtype == FD_F64 ? backward_bytes<double>(m, p, algo) : backward_bytes<float>(m, p, algo);
    return FD_OK;
}

fd_status_t fd_backward(const fd_model_t* m, const fd_batch_t* b, const void* q, const void* qd, const void* tau,
                        const void* qdd, const void* gqdd, void* gq, void* gqd, void* gtau, fd_algo_t algo,
                        int accumulate, void* ws, size_t ws_bytes, void* hip_stream) {
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (algo < FD_ALGO_ABIA || algo > FD_ALGO_CFA_PROJ) return FD_ERR_INVALID_ARG;
    if (b->batch == 0) return FD_OK;
    if (!q || !qd || (!qdd && !tau) || !gqdd || !gq || !gqd || !gtau) return FD_ERR_INVALID_ARG;
    algo = backward_algo(m, p, b->batch, algo);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (m->dtype == FD_F64)
        return backward_t<double>(m, p, q, qd, tau, qdd, gqdd, gq, gqd, gtau, algo, accumulate, ws, ws_bytes, st);
    return backward_t<float>(m, p, q, qd, tau, qdd, gqdd, gq, gqd, gtau, algo, accumulate, ws, ws_bytes, st);
}

fd_status_t fd_euler_step(fd_dtype_t dtype, int64_t count, double dt, const void* q, const void* qd, const void* qdd,
                          void* qn, void* qdn, void* hip_stream) {
    if ((dtype != FD_F64 && dtype != FD_F32) || count < 0 || !std::isfinite(dt)) return FD_ERR_INVALID_ARG;
    if (count == 0) return FD_OK;
    if (!q || !qd || !qdd || !qn || !qdn) return FD_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (dtype == FD_F64)
        return from_hip(fdk::launch_euler<double>(count, dt, (const double*)q, (const double*)qd, (const double*)qdd,
                                                  (double*)qn, (double*)qdn, st));
    return from_hip(fdk::launch_euler<float>(count, (float)dt, (const float*)q, (const float*)qd, (const float*)qdd,
                                             (float*)qn, (float*)qdn, st));
}

fd_status_t fd_euler_step_backward(fd_dtype_t dtype, int64_t count, double dt, const void* gqn, const void* gqdn,
                                   void* gq, void* gqd, void* gqdd, void* hip_stream) {
    if ((dtype != FD_F64 && dtype != FD_F32) || count < 0 || !std::isfinite(dt)) return FD_ERR_INVALID_ARG;
    if (count == 0) return FD_OK;
    if (!gqn || !gqdn || !gq || !gqd || !gqdd) return FD_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (dtype == FD_F64)
        return from_hip(fdk::launch_euler_vjp<double>(count, dt, (const double*)gqn, (const double*)gqdn, (double*)gq,
                                                      (double*)gqd, (double*)gqdd, st));
    return from_hip(fdk::launch_euler_vjp<float>(count, (float)dt, (const float*)gqn, (const float*)gqdn, (float*)gq,
                                                 (float*)gqd, (float*)gqdd, st));
}

fd_status_t fd_inverse(const fd_model_t* m, const fd_batch_t* b, const void* q, const void* qd, const void* qdd,
                       int gravity, void* tau, void* hip_stream) {
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (m->tree && !m->depth_first) return FD_ERR_UNSUPPORTED;
    if (b->batch == 0) return FD_OK;
    if (!q || !qd || !tau) return FD_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int np = pow2_lanes(p.nmax);
    if (m->dtype == FD_F64)
        return from_hip(fdk::launch_inverse<double>(np, view<double>(m), p.cm, (const double*)q, (const double*)qd,
                                                    (const double*)qdd, gravity, (double*)tau, st));
    return from_hip(fdk::launch_inverse<float>(np, view<float>(m), p.cm, (const float*)q, (const float*)qd,
                                               (const float*)qdd, gravity, (float*)tau, st));
}

fd_status_t fd_joint_inertia(const fd_model_t* m, const fd_batch_t* b, const void* q, void* m_out, void* hip_stream) {
    BatchPlan p;
    fd_status_t s = plan_batch(m, b, &p);
    if (s != FD_OK) return s;
    if (m->tree && !m->depth_first) return FD_ERR_UNSUPPORTED;
    if (b->offsets != nullptr) return FD_ERR_INVALID_ARG;
    if (b->batch == 0) return FD_OK;
    if (!q || !m_out) return FD_ERR_INVALID_ARG;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int np = pow2_lanes(p.nmax);
    if (m->dtype == FD_F64)
        return from_hip(fdk::launch_mass<double>(np, view<double>(m), p.cm, (const double*)q, (double*)m_out, st));
    return from_hip(fdk::launch_mass<float>(np, view<float>(m), p.cm, (const float*)q, (float*)m_out, st));
}

fd_status_t fd_scan6(fd_dtype_t dtype, int32_t segs, const int64_t* off, int32_t max_len, const void* b,
                     const void* c, int reverse, void* x, void* hip_stream) {
    if (segs < 0 || (dtype != FD_F64 && dtype != FD_F32)) return FD_ERR_INVALID_ARG;
    if (segs == 0) return FD_OK;
    if (!off || !b || !c || !x || max_len < 1) return FD_ERR_INVALID_ARG;
    if (max_len > kMaxLinks) return FD_ERR_UNSUPPORTED;
    const int np = pow2_lanes(max_len);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (dtype == FD_F64)
        return from_hip(fdk::launch_scan6<double>(np, segs, off, (const double*)b, (const double*)c, reverse,
                                                  (double*)x, st));
    return from_hip(fdk::launch_scan6<float>(np, segs, off, (const float*)b, (const float*)c, reverse, (float*)x, st));
}

fd_status_t fd_btd_solve6(fd_dtype_t dtype, int32_t segs, const int64_t* off, int32_t max_len, const void* d,
                          const void* u, const void* r, void* x, int* status, void* hip_stream) {
    if (segs < 0 || (dtype != FD_F64 && dtype != FD_F32)) return FD_ERR_INVALID_ARG;
    if (segs == 0) return FD_OK;
    if (!off || !d || !u || !r || !x || max_len < 1) return FD_ERR_INVALID_ARG;
    if (max_len > kMaxLinks) return FD_ERR_UNSUPPORTED;
    const int np = pow2_lanes(max_len);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (dtype == FD_F64)
        return from_hip(fdk::launch_btd6<double>(np, segs, off, (const double*)d, (const double*)u, (const double*)r,
                                                 (double*)x, status, st));
    return from_hip(fdk::launch_btd6<float>(np, segs, off, (const float*)d, (const float*)u, (const float*)r,
                                            (float*)x, status, st));
}

fd_status_t fd_set_auto_table(fd_dtype_t dtype, const int8_t* table) {
    if (dtype != FD_F64 && dtype != FD_F32) return FD_ERR_INVALID_ARG;
    std::vector<int8_t>& t = g_auto[dtype == FD_F64 ? 0 : 1];
    if (!table) {
        t.clear();
        return FD_OK;
    }
    std::vector<int8_t> next(table, table + 257 * 21);
    const int jmax = dtype == FD_F64 ? fdk::jsiia_max_np<double>() : fdk::jsiia_max_np<float>();
    for (int n = 1; n <= kMaxLinks; ++n)
        for (int k = 0; k < 21; ++k) {
            int a = next[n * 21 + k];
            if (a < FD_ALGO_ABIA || a > FD_ALGO_CFA_PROJ || a == FD_ALGO_AUTO) return FD_ERR_INVALID_ARG;
            if (a == FD_ALGO_JSIIA && pow2_lanes(n) > jmax) return FD_ERR_INVALID_ARG;
        }
    t.swap(next);
    return FD_OK;
}

fd_status_t fd_set_persistent_grid(fd_dtype_t dtype, int32_t grid) {
    if ((dtype != FD_F64 && dtype != FD_F32) || grid < 0) return FD_ERR_INVALID_ARG;
    g_persistent_grid[dtype == FD_F64 ? 0 : 1] = grid;
    return FD_OK;
}

const char* fd_status_string(fd_status_t s) {
    switch (s) {
        case FD_OK: return "ok";
        case FD_ERR_INVALID_ARG: return "invalid argument";
        case FD_ERR_UNSUPPORTED: return "unsupported by this library";
        case FD_ERR_OUT_OF_MEMORY: return "out of device memory";
        case FD_ERR_DEVICE: return "device error";
        case FD_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

}  // extern "C"
