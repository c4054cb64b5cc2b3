/*
 * fd_oracle.c -- plain, slow CPU oracle for forward dynamics of serial chains.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may link,
 * load or call this file: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code, header or constant with the HIP
 * path.
 *
 * What it computes is the plain definition of forward dynamics (Sec. II-C,
 * eq. (eq-motion) and (tau-bias)):
 *
 *     qdd = M(q)^-1 (tau - tau_bias(q, qd)),
 *
 * with M built by the composite-rigid-body method, tau_bias by recursive
 * Newton-Euler at qdd = 0 (gravity included), and the solve by a dense
 * Cholesky factorisation.  All three algorithms of the paper (JSIIA, ABIA,
 * CFA) reach exactly this value in exact arithmetic.
 *
 * Conventions (the paper leaves them open; this is the reading taken):
 *   twist V = (w; v), wrench F = (n; f), [a] = 3x3 cross-product matrix;
 *   Ad_T = [[R, 0], [[p]R, R]] for a pose T = (R, p);
 *   ad_V = [[[w], 0], [[v], [w]]], and ad*_V is ad_V^T (Sec. II-A);
 *   spatial inertia about the frame origin
 *       J = [[Ic - m[c][c], m[c]], [-m[c], m 1]];
 *   joint i: T_{i-1,i} = (Rhome_i Rot(axis_i, q_i), offset_i), S_i = (axis_i; 0);
 *   Ad_i = Ad(T_{i-1,i}^-1) maps frame i-1 twists into frame i (the (i, i-1)
 *   block of Gamma in eq. (EOM-full));
 *   base twist V_0 = 0, base acceleration (0; -g) (gravity as a fictitious
 *   base acceleration, the "const." terms of eq. (EOM-full)), tip force 0.
 *
 * Recursions (eq. (EOM-single) applied link by link, eq. (EOM-full)):
 *   V_i  = Ad_i V_{i-1} + S_i qd_i
 *   A_i  = Ad_i A_{i-1} + S_i qdd_i + ad_{V_i}(S_i qd_i)
 *   F_i  = Ad_{i+1}^T F_{i+1} + J_i A_i - ad_{V_i}^T (J_i V_i)
 *   tau_i = S_i^T F_i
 *
 * Everything is written with explicit 6x6 matrices so that it can be checked
 * against the formulas by eye; speed is not a goal.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double a[6][6]; } mat6;
typedef struct { double a[6]; } vec6;

typedef struct {
    int n;
    const double *axis, *home_rot, *offset, *mass, *com, *inertia;
    double g[3];
} chain_t;

/* ---------- small dense helpers ---------- */

static void skew3(const double v[3], double s[3][3]) {
    s[0][0] = 0;     s[0][1] = -v[2]; s[0][2] = v[1];
    s[1][0] = v[2];  s[1][1] = 0;     s[1][2] = -v[0];
    s[2][0] = -v[1]; s[2][1] = v[0];  s[2][2] = 0;
}

static void mul3(const double a[3][3], const double b[3][3], double c[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += a[i][k] * b[k][j];
            c[i][j] = s;
        }
}

static mat6 mat6_zero(void) { mat6 m; memset(&m, 0, sizeof m); return m; }

static mat6 mat6_mul(const mat6 *a, const mat6 *b) {
    mat6 c;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += a->a[i][k] * b->a[k][j];
            c.a[i][j] = s;
        }
    return c;
}

static mat6 mat6_tr(const mat6 *a) {
    mat6 c;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) c.a[i][j] = a->a[j][i];
    return c;
}

static mat6 mat6_add(const mat6 *a, const mat6 *b) {
    mat6 c;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) c.a[i][j] = a->a[i][j] + b->a[i][j];
    return c;
}

static vec6 mat6_vec(const mat6 *a, const vec6 *x) {
    vec6 y;
    for (int i = 0; i < 6; ++i) {
        double s = 0;
        for (int k = 0; k < 6; ++k) s += a->a[i][k] * x->a[k];
        y.a[i] = s;
    }
    return y;
}

static vec6 vec6_add(const vec6 *a, const vec6 *b) {
    vec6 c;
    for (int i = 0; i < 6; ++i) c.a[i] = a->a[i] + b->a[i];
    return c;
}

static vec6 vec6_sub(const vec6 *a, const vec6 *b) {
    vec6 c;
    for (int i = 0; i < 6; ++i) c.a[i] = a->a[i] - b->a[i];
    return c;
}

static vec6 vec6_scale(const vec6 *a, double s) {
    vec6 c;
    for (int i = 0; i < 6; ++i) c.a[i] = a->a[i] * s;
    return c;
}

static double vec6_dot(const vec6 *a, const vec6 *b) {
    double s = 0;
    for (int i = 0; i < 6; ++i) s += a->a[i] * b->a[i];
    return s;
}

/* ---------- Lie-group quantities (Sec. II-A) ---------- */

/* Rot(w, q) = I + sin q [w] + (1 - cos q) [w]^2 for a unit axis w. */
static void rot_axis_angle(const double w[3], double q, double r[3][3]) {
    double k[3][3], k2[3][3];
    skew3(w, k);
    mul3(k, k, k2);
    double s = sin(q), c = 1.0 - cos(q);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) r[i][j] = (i == j ? 1.0 : 0.0) + s * k[i][j] + c * k2[i][j];
}

/* Pose of frame i in frame i-1: T_{i-1,i} = (Rhome Rot(axis, q), offset). */
static void link_pose(const chain_t *c, int i, double q, double r[3][3], double p[3]) {
    double rh[3][3], rq[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) rh[a][b] = c->home_rot[9 * i + 3 * a + b];
    rot_axis_angle(&c->axis[3 * i], q, rq);
    mul3(rh, rq, r);
    for (int a = 0; a < 3; ++a) p[a] = c->offset[3 * i + a];
}

/* Ad_T = [[R, 0], [[p]R, R]]. */
static mat6 ad_pose(const double r[3][3], const double p[3]) {
    double s[3][3], pr[3][3];
    skew3(p, s);
    mul3(s, r, pr);
    mat6 m = mat6_zero();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            m.a[i][j] = r[i][j];
            m.a[i + 3][j + 3] = r[i][j];
            m.a[i + 3][j] = pr[i][j];
        }
    return m;
}

/* Ad of the inverse pose (R^T, -R^T p). */
static mat6 ad_pose_inv(const double r[3][3], const double p[3]) {
    double rt[3][3], pi[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) rt[i][j] = r[j][i];
    for (int i = 0; i < 3; ++i) pi[i] = -(rt[i][0] * p[0] + rt[i][1] * p[1] + rt[i][2] * p[2]);
    return ad_pose(rt, pi);
}

/* ad_V = [[[w], 0], [[v], [w]]]. */
static mat6 ad_twist(const vec6 *v) {
    double w[3] = {v->a[0], v->a[1], v->a[2]}, u[3] = {v->a[3], v->a[4], v->a[5]};
    double sw[3][3], su[3][3];
    skew3(w, sw);
    skew3(u, su);
    mat6 m = mat6_zero();
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            m.a[i][j] = sw[i][j];
            m.a[i + 3][j + 3] = sw[i][j];
            m.a[i + 3][j] = su[i][j];
        }
    return m;
}

/* J = [[Ic - m[c][c], m[c]], [-m[c], m 1]] about the frame origin. */
static mat6 spatial_inertia(const chain_t *c, int i) {
    double m = c->mass[i];
    const double *cc = &c->com[3 * i];
    const double *in = &c->inertia[6 * i];
    double ic[3][3] = {{in[0], in[3], in[4]}, {in[3], in[1], in[5]}, {in[4], in[5], in[2]}};
    double sc[3][3], sc2[3][3];
    skew3(cc, sc);
    mul3(sc, sc, sc2);
    mat6 j = mat6_zero();
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            j.a[a][b] = ic[a][b] - m * sc2[a][b];
            j.a[a][b + 3] = m * sc[a][b];
            j.a[a + 3][b] = -m * sc[a][b];
        }
    for (int a = 0; a < 3; ++a) j.a[a + 3][a + 3] = m;
    return j;
}

static vec6 joint_screw(const chain_t *c, int i) {
    vec6 s = {{c->axis[3 * i], c->axis[3 * i + 1], c->axis[3 * i + 2], 0, 0, 0}};
    return s;
}

/* ---------- recursive Newton-Euler (eq. (EOM-full), qdd given) ---------- */

static void rnea_chain(const chain_t *c, const double *q, const double *qd, const double *qdd,
                       int with_gravity, double *tau, vec6 *work_v, vec6 *work_f, mat6 *work_ad) {
    int n = c->n;
    vec6 vprev = {{0, 0, 0, 0, 0, 0}};
    vec6 aprev = {{0, 0, 0, 0, 0, 0}};
    if (with_gravity) {
        aprev.a[3] = -c->g[0];
        aprev.a[4] = -c->g[1];
        aprev.a[5] = -c->g[2];
    }
    for (int i = 0; i < n; ++i) {
        double r[3][3], p[3];
        link_pose(c, i, q[i], r, p);
        work_ad[i] = ad_pose_inv(r, p);
        vec6 s = joint_screw(c, i);
        vec6 sqd = vec6_scale(&s, qd[i]);
        vec6 t = mat6_vec(&work_ad[i], &vprev);
        vec6 v = vec6_add(&t, &sqd);
        mat6 adv = ad_twist(&v);
        vec6 corr = mat6_vec(&adv, &sqd);
        vec6 ta = mat6_vec(&work_ad[i], &aprev);
        vec6 sqdd = vec6_scale(&s, qdd ? qdd[i] : 0.0);
        vec6 a = vec6_add(&ta, &sqdd);
        a = vec6_add(&a, &corr);
        mat6 j = spatial_inertia(c, i);
        vec6 jv = mat6_vec(&j, &v);
        vec6 ja = mat6_vec(&j, &a);
        mat6 advt = mat6_tr(&adv);
        vec6 gyro = mat6_vec(&advt, &jv);
        work_f[i] = vec6_sub(&ja, &gyro);
        work_v[i] = v;
        vprev = v;
        aprev = a;
    }
    vec6 fnext = {{0, 0, 0, 0, 0, 0}};
    for (int i = n - 1; i >= 0; --i) {
        vec6 f = work_f[i];
        if (i + 1 < n) {
            mat6 adt = mat6_tr(&work_ad[i + 1]);
            vec6 t = mat6_vec(&adt, &fnext);
            f = vec6_add(&f, &t);
        }
        vec6 s = joint_screw(c, i);
        tau[i] = vec6_dot(&s, &f);
        fnext = f;
    }
}

/* ---------- composite-rigid-body joint-space inertia ---------- */

static void crba_chain(const chain_t *c, const double *q, double *m_out, mat6 *work_ad, mat6 *work_ic) {
    int n = c->n;
    for (int i = 0; i < n; ++i) {
        double r[3][3], p[3];
        link_pose(c, i, q[i], r, p);
        work_ad[i] = ad_pose_inv(r, p);
    }
    /* Ic_n = J_n; Ic_i = J_i + Ad_{i+1}^T Ic_{i+1} Ad_{i+1} */
    for (int i = n - 1; i >= 0; --i) {
        work_ic[i] = spatial_inertia(c, i);
        if (i + 1 < n) {
            mat6 adt = mat6_tr(&work_ad[i + 1]);
            mat6 t = mat6_mul(&adt, &work_ic[i + 1]);
            mat6 t2 = mat6_mul(&t, &work_ad[i + 1]);
            work_ic[i] = mat6_add(&work_ic[i], &t2);
        }
    }
    for (int i = 0; i < n; ++i) {
        vec6 si = joint_screw(c, i);
        vec6 f = mat6_vec(&work_ic[i], &si);
        m_out[i * n + i] = vec6_dot(&si, &f);
        for (int j = i; j >= 1; --j) {
            mat6 adt = mat6_tr(&work_ad[j]);
            f = mat6_vec(&adt, &f);
            vec6 sj = joint_screw(c, j - 1);
            double v = vec6_dot(&sj, &f);
            m_out[(j - 1) * n + i] = v;
            m_out[i * n + (j - 1)] = v;
        }
    }
}

/* ---------- dense Cholesky solve M x = b (no pivoting; M must be SPD) ---------- */

static int cholesky_solve(int n, double *m, const double *b, double *x) {
    /* in-place lower factor in m (row-major) */
    for (int j = 0; j < n; ++j) {
        double d = m[j * n + j];
        for (int k = 0; k < j; ++k) d -= m[j * n + k] * m[j * n + k];
        if (!(d > 0.0)) return -1;
        double ljj = sqrt(d);
        m[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = m[i * n + j];
            for (int k = 0; k < j; ++k) s -= m[i * n + k] * m[j * n + k];
            m[i * n + j] = s / ljj;
        }
    }
    for (int i = 0; i < n; ++i) {          /* L y = b */
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= m[i * n + k] * x[k];
        x[i] = s / m[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {     /* L^T x = y */
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= m[k * n + i] * x[k];
        x[i] = s / m[i * n + i];
    }
    return 0;
}

/* ---------- forward kinematics and energy ---------- */

static void fk_chain(const chain_t *c, const double *q, double *rot_out, double *pos_out) {
    double racc[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, pacc[3] = {0, 0, 0};
    for (int i = 0; i < c->n; ++i) {
        double r[3][3], p[3], rn[3][3], pn[3];
        link_pose(c, i, q[i], r, p);
        mul3(racc, r, rn);
        for (int a = 0; a < 3; ++a)
            pn[a] = pacc[a] + racc[a][0] * p[0] + racc[a][1] * p[1] + racc[a][2] * p[2];
        memcpy(racc, rn, sizeof racc);
        memcpy(pacc, pn, sizeof pacc);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) rot_out[9 * i + 3 * a + b] = racc[a][b];
        for (int a = 0; a < 3; ++a) pos_out[3 * i + a] = pacc[a];
    }
}

/* ---------- chain view from packed arrays ---------- */

typedef struct {
    const double *axis, *home_rot, *offset, *mass, *com, *inertia, *gravity;
} model_arrays_t;

static chain_t chain_at(const model_arrays_t *ma, int64_t start, int n) {
    chain_t c;
    c.n = n;
    c.axis = ma->axis + 3 * start;
    c.home_rot = ma->home_rot + 9 * start;
    c.offset = ma->offset + 3 * start;
    c.mass = ma->mass + start;
    c.com = ma->com + 3 * start;
    c.inertia = ma->inertia + 6 * start;
    for (int a = 0; a < 3; ++a) c.g[a] = ma->gravity[a];
    return c;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    omp_set_num_threads(nthreads > 0 ? nthreads : omp_get_num_procs());
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define MODEL_ARGS                                                                          \
    const double *axis, const double *home_rot, const double *offset, const double *mass,   \
        const double *com, const double *inertia, const double *gravity
#define MODEL_INIT model_arrays_t ma = {axis, home_rot, offset, mass, com, inertia, gravity}
#define MSTART(b) (model_start ? model_start[b] : offsets[b])

/*
 * Inverse dynamics: tau = ID(q, qd, qdd) for every chain (qdd may be NULL = 0).
 * offsets[batch+1]: chain b owns state entries [offsets[b], offsets[b+1]).
 * model_start[batch] (or NULL = offsets): first link of chain b's robot.
 */
int oracle_rnea_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                      const double *q, const double *qd, const double *qdd, int with_gravity,
                      double *tau, int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) continue;
        chain_t c = chain_at(&ma, MSTART(b), n);
        vec6 *wv = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n);
        if (!wv || !wf || !wa) { bad++; free(wv); free(wf); free(wa); continue; }
        int64_t o = offsets[b];
        rnea_chain(&c, q + o, qd + o, qdd ? qdd + o : NULL, with_gravity, tau + o, wv, wf, wa);
        free(wv); free(wf); free(wa);
    }
    return bad ? -1 : 0;
}

/* Joint-space inertia of every chain; chain b's n*n block starts at m_start[b]. */
int oracle_crba_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                      const double *q, const int64_t *m_start, double *m_out, int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) continue;
        chain_t c = chain_at(&ma, MSTART(b), n);
        mat6 *wa = malloc(sizeof(mat6) * n), *wi = malloc(sizeof(mat6) * n);
        if (!wa || !wi) { bad++; free(wa); free(wi); continue; }
        crba_chain(&c, q + offsets[b], m_out + m_start[b], wa, wi);
        free(wa); free(wi);
    }
    return bad ? -1 : 0;
}

/*
 * Forward dynamics by the plain definition: qdd = M^-1 (tau - ID(q, qd, 0)).
 * Returns the number of chains whose M was not numerically SPD (their qdd is NaN).
 */
int oracle_fd_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                    const double *q, const double *qd, const double *tau, double *qdd, int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) continue;
        int64_t o = offsets[b];
        chain_t c = chain_at(&ma, MSTART(b), n);
        vec6 *wv = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n), *wi = malloc(sizeof(mat6) * n);
        double *m = malloc(sizeof(double) * n * n), *bias = malloc(sizeof(double) * n);
        if (!wv || !wf || !wa || !wi || !m || !bias) {
            bad++;
        } else {
            rnea_chain(&c, q + o, qd + o, NULL, 1, bias, wv, wf, wa);
            for (int i = 0; i < n; ++i) bias[i] = tau[o + i] - bias[i];
            crba_chain(&c, q + o, m, wa, wi);
            if (cholesky_solve(n, m, bias, qdd + o) != 0) {
                bad++;
                for (int i = 0; i < n; ++i) qdd[o + i] = NAN;
            }
        }
        free(wv); free(wf); free(wa); free(wi); free(m); free(bias);
    }
    return bad;
}

/* Base-frame pose of every link: rot [N][9] row-major, pos [N][3]. */
int oracle_fk_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                    const double *q, double *rot, double *pos, int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) continue;
        int64_t o = offsets[b];
        chain_t c = chain_at(&ma, MSTART(b), n);
        fk_chain(&c, q + o, rot + 9 * o, pos + 3 * o);
    }
    return 0;
}

/*
 * Mechanical energy of every chain: kinetic 1/2 sum V_i^T J_i V_i (body twists
 * from the forward velocity recursion) and potential -sum m_i g . x_com,i.
 */
int oracle_energy_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                        const double *q, const double *qd, double *kinetic, double *potential,
                        int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) { kinetic[b] = 0; potential[b] = 0; continue; }
        int64_t o = offsets[b];
        chain_t c = chain_at(&ma, MSTART(b), n);
        double *rot = malloc(sizeof(double) * 9 * n), *pos = malloc(sizeof(double) * 3 * n);
        if (!rot || !pos) { bad++; free(rot); free(pos); continue; }
        fk_chain(&c, q + o, rot, pos);
        double ke = 0, pe = 0;
        vec6 vprev = {{0, 0, 0, 0, 0, 0}};
        for (int i = 0; i < n; ++i) {
            double r[3][3], p[3];
            link_pose(&c, i, q[o + i], r, p);
            mat6 ad = ad_pose_inv(r, p);
            vec6 s = joint_screw(&c, i);
            vec6 sqd = vec6_scale(&s, qd[o + i]);
            vec6 t = mat6_vec(&ad, &vprev);
            vec6 v = vec6_add(&t, &sqd);
            mat6 j = spatial_inertia(&c, i);
            vec6 jv = mat6_vec(&j, &v);
            ke += 0.5 * vec6_dot(&v, &jv);
            vprev = v;
            const double *cc = &c.com[3 * i];
            double xc[3];
            for (int a = 0; a < 3; ++a)
                xc[a] = pos[3 * i + a] + rot[9 * i + 3 * a] * cc[0] + rot[9 * i + 3 * a + 1] * cc[1] +
                        rot[9 * i + 3 * a + 2] * cc[2];
            pe -= c.mass[i] * (c.g[0] * xc[0] + c.g[1] * xc[1] + c.g[2] * xc[2]);
        }
        kinetic[b] = ke;
        potential[b] = pe;
        free(rot); free(pos);
    }
    return bad ? -1 : 0;
}

/* Single-link helpers for the property tests of the Lie-group primitives. */
void oracle_link_rotation(const double *axis, const double *home_rot, double q, double *r_out) {
    chain_t c;
    memset(&c, 0, sizeof c);
    double off[3] = {0, 0, 0};
    c.n = 1;
    c.axis = axis;
    c.home_rot = home_rot;
    c.offset = off;
    double r[3][3], p[3];
    link_pose(&c, 0, q, r, p);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) r_out[3 * a + b] = r[a][b];
}

void oracle_adjoint(const double *rot, const double *pos, int inverse, double *out) {
    double r[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) r[a][b] = rot[3 * a + b];
    mat6 m = inverse ? ad_pose_inv(r, pos) : ad_pose(r, pos);
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) out[6 * a + b] = m.a[a][b];
}

void oracle_spatial_inertia(double mass, const double *com, const double *inertia, double *out) {
    chain_t c;
    memset(&c, 0, sizeof c);
    c.n = 1;
    c.mass = &mass;
    c.com = com;
    c.inertia = inertia;
    mat6 j = spatial_inertia(&c, 0);
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) out[6 * a + b] = j.a[a][b];
}
