/*
 * fd_oracle.c -- plain, slow CPU oracle for forward dynamics of serial chains
 * (and of branched trees).
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
 * Branched robots (trees; the paper treats serial chains only). Link i hangs
 * from link p(i) < i, or from the base, and its pose is taken in p(i)'s frame:
 * Gamma has the block Ad_i at (i, p(i)) instead of (i, i - 1). Then i - 1
 * above reads p(i), and F_i sums Ad_c^T F_c over all children c of i.
 *
 * Everything is written with explicit 6x6 matrices so that it can be checked
 * against the formulas by eye; speed is not a goal.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fd_chain.h"



#define REAL double
#define RSIN sin
#define RCOS cos
#define RSQRT sqrt
#define RE(x) (x)
#include "fd_core.inc"

/* ---------- chain view from packed arrays ---------- */

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}



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
        vec6 *wv = malloc(sizeof(vec6) * n), *wc = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n);
        if (!wv || !wc || !wf || !wa) { bad++; free(wv); free(wc); free(wf); free(wa); continue; }
        int64_t o = offsets[b];
        rnea_chain(&c, q + o, qd + o, qdd ? qdd + o : NULL, with_gravity, tau + o, wv, wc, wf, wa);
        free(wv); free(wc); free(wf); free(wa);
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
        vec6 *wv = malloc(sizeof(vec6) * n), *wc = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n), *wi = malloc(sizeof(mat6) * n);
        double *m = malloc(sizeof(double) * n * n), *bias = malloc(sizeof(double) * n);
        if (!wv || !wc || !wf || !wa || !wi || !m || !bias) {
            bad++;
        } else {
            rnea_chain(&c, q + o, qd + o, NULL, 1, bias, wv, wc, wf, wa);
            for (int i = 0; i < n; ++i) bias[i] = tau[o + i] - bias[i];
            crba_chain(&c, q + o, m, wa, wi);
            if (cholesky_solve(n, m, bias, qdd + o) != 0) {
                bad++;
                for (int i = 0; i < n; ++i) qdd[o + i] = NAN;
            }
        }
        free(wv); free(wc); free(wf); free(wa); free(wi); free(m); free(bias);
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
        vec6 *vl = malloc(sizeof(vec6) * n);
        if (!rot || !pos || !vl) { bad++; free(rot); free(pos); free(vl); continue; }
        fk_chain(&c, q + o, rot, pos);
        double ke = 0, pe = 0;
        vec6 vbase = {{0, 0, 0, 0, 0, 0}};
        for (int i = 0; i < n; ++i) {
            double r[3][3], p[3];
            link_pose(&c, i, q[o + i], r, p);
            mat6 ad = ad_pose_inv(r, p);
            vec6 s = joint_screw(&c, i);
            vec6 sqd = vec6_scale(&s, qd[o + i]);
            int par = parent_of(&c, i);
            vec6 t = mat6_vec(&ad, par >= 0 ? &vl[par] : &vbase);
            vec6 v = vec6_add(&t, &sqd);
            mat6 j = spatial_inertia(&c, i);
            vec6 jv = mat6_vec(&j, &v);
            ke += 0.5 * vec6_dot(&v, &jv);
            vl[i] = v;
            const double *cc = &c.com[3 * i];
            double xc[3];
            for (int a = 0; a < 3; ++a)
                xc[a] = pos[3 * i + a] + rot[9 * i + 3 * a] * cc[0] + rot[9 * i + 3 * a + 1] * cc[1] +
                        rot[9 * i + 3 * a + 2] * cc[2];
            pe -= c.mass[i] * (c.g[0] * xc[0] + c.g[1] * xc[1] + c.g[2] * xc[2]);
        }
        kinetic[b] = ke;
        potential[b] = pe;
        free(rot); free(pos); free(vl);
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
