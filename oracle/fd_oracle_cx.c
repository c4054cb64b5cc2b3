/*
 * fd_oracle_cx.c -- directional derivatives of the oracle by the complex step.
 *
 * TEST INFRASTRUCTURE ONLY (see fd_oracle.c). The same arithmetic as the
 * oracle (fd_core.inc) evaluated in double complex: with inputs x + i h v,
 * Im f / h is the derivative of f along v to rounding (no subtractive
 * cancellation), for h far below the scale of x. It checks the adjoint of
 * forward dynamics by the identity <VJP(g), v> = <g, JVP(v)>.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fd_chain.h"

#define REAL double complex
#define RSIN csin
#define RCOS ccos
#define RSQRT csqrt
#define RE(x) creal(x)
#include "fd_core.inc"

#define CX_STEP 1e-30

/*
 * d qdd along (dq, dqd, dtau) for every chain: qdd = M(q)^-1 (tau - ID(q, qd, 0)).
 * Also writes qdd itself. Returns the number of chains whose M was not SPD.
 */
int oracle_fd_jvp_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                        const double *q, const double *qd, const double *tau, const double *dq,
                        const double *dqd, const double *dtau, double *qdd, double *dqdd, int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) continue;
        int64_t o = offsets[b];
        chain_t c = chain_at(&ma, MSTART(b), n);
        REAL *xq = malloc(sizeof(REAL) * n), *xqd = malloc(sizeof(REAL) * n), *xt = malloc(sizeof(REAL) * n);
        REAL *bias = malloc(sizeof(REAL) * n), *x = malloc(sizeof(REAL) * n), *m = malloc(sizeof(REAL) * n * n);
        vec6 *wv = malloc(sizeof(vec6) * n), *wc = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n), *wi = malloc(sizeof(mat6) * n);
        if (!xq || !xqd || !xt || !bias || !x || !m || !wv || !wc || !wf || !wa || !wi) {
            bad++;
        } else {
            for (int i = 0; i < n; ++i) {
                xq[i] = q[o + i] + I * CX_STEP * dq[o + i];
                xqd[i] = qd[o + i] + I * CX_STEP * dqd[o + i];
                xt[i] = tau[o + i] + I * CX_STEP * dtau[o + i];
            }
            rnea_chain(&c, xq, xqd, NULL, 1, bias, wv, wc, wf, wa);
            for (int i = 0; i < n; ++i) bias[i] = xt[i] - bias[i];
            crba_chain(&c, xq, m, wa, wi);
            if (cholesky_solve(n, m, bias, x) != 0) {
                bad++;
                for (int i = 0; i < n; ++i) { qdd[o + i] = NAN; dqdd[o + i] = NAN; }
            } else {
                for (int i = 0; i < n; ++i) {
                    qdd[o + i] = creal(x[i]);
                    dqdd[o + i] = cimag(x[i]) / CX_STEP;
                }
            }
        }
        free(xq); free(xqd); free(xt); free(bias); free(x); free(m); free(wv); free(wc); free(wf); free(wa); free(wi);
    }
    return bad;
}

/* d tau along (dq, dqd, dqdd) of the inverse dynamics tau = ID(q, qd, qdd). */
int oracle_rnea_jvp_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
                          const double *q, const double *qd, const double *qdd, const double *dq,
                          const double *dqd, const double *dqdd, int with_gravity, double *dtau, int nthreads) {
    MODEL_INIT;
    set_threads(nthreads);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int b = 0; b < batch; ++b) {
        int n = (int)(offsets[b + 1] - offsets[b]);
        if (n <= 0) continue;
        int64_t o = offsets[b];
        chain_t c = chain_at(&ma, MSTART(b), n);
        REAL *xq = malloc(sizeof(REAL) * n), *xqd = malloc(sizeof(REAL) * n), *xa = malloc(sizeof(REAL) * n);
        REAL *t = malloc(sizeof(REAL) * n);
        vec6 *wv = malloc(sizeof(vec6) * n), *wc = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n);
        if (!xq || !xqd || !xa || !t || !wv || !wc || !wf || !wa) {
            bad++;
        } else {
            for (int i = 0; i < n; ++i) {
                xq[i] = q[o + i] + I * CX_STEP * dq[o + i];
                xqd[i] = qd[o + i] + I * CX_STEP * dqd[o + i];
                xa[i] = qdd[o + i] + I * CX_STEP * dqdd[o + i];
            }
            rnea_chain(&c, xq, xqd, xa, with_gravity, t, wv, wc, wf, wa);
            for (int i = 0; i < n; ++i) dtau[o + i] = cimag(t[i]) / CX_STEP;
        }
        free(xq); free(xqd); free(xa); free(t); free(wv); free(wc); free(wf); free(wa);
    }
    return bad ? -1 : 0;
}
