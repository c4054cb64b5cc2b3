/*
 * fd_oracle_ld.c -- the oracle's forward dynamics in extended precision.
 *
 * TEST INFRASTRUCTURE ONLY (see fd_oracle.c). The same arithmetic as the
 * oracle (fd_core.inc) evaluated in long double (the x87 80-bit format on
 * x86-64: a 64-bit significand, unit roundoff 2^-64 = 5.4e-20), with the model
 * parameters and the joint states taken exactly as given in double. Its
 * rounding error is below 2^-11 of the double evaluation's, so it serves as
 * the exact reference of a forward-dynamics result: in double, the oracle's
 * own error grows as cond(M) u and reaches 1e-10 on long, ill-conditioned
 * chains, where it would otherwise be counted against the GPU result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "fd_chain.h"

#define REAL long double
#define RSIN sinl
#define RCOS cosl
#define RSQRT sqrtl
#define RE(x) (x)
#include "fd_core.inc"

/* qdd = M^-1 (tau - ID(q, qd, 0)) in long double, rounded to double at the end. */
int oracle_fd_ld_batch(int batch, const int64_t *offsets, const int64_t *model_start, MODEL_ARGS,
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
        REAL *xq = malloc(sizeof(REAL) * n), *xqd = malloc(sizeof(REAL) * n), *bias = malloc(sizeof(REAL) * n);
        REAL *x = malloc(sizeof(REAL) * n), *m = malloc(sizeof(REAL) * n * n);
        vec6 *wv = malloc(sizeof(vec6) * n), *wc = malloc(sizeof(vec6) * n), *wf = malloc(sizeof(vec6) * n);
        mat6 *wa = malloc(sizeof(mat6) * n), *wi = malloc(sizeof(mat6) * n);
        if (!xq || !xqd || !bias || !x || !m || !wv || !wc || !wf || !wa || !wi) {
            bad++;
        } else {
            for (int i = 0; i < n; ++i) {
                xq[i] = q[o + i];
                xqd[i] = qd[o + i];
            }
            rnea_chain(&c, xq, xqd, NULL, 1, bias, wv, wc, wf, wa);
            for (int i = 0; i < n; ++i) bias[i] = (REAL)tau[o + i] - bias[i];
            crba_chain(&c, xq, m, wa, wi);
            if (cholesky_solve(n, m, bias, x) != 0) {
                bad++;
                for (int i = 0; i < n; ++i) qdd[o + i] = NAN;
            } else {
                for (int i = 0; i < n; ++i) qdd[o + i] = (double)x[i];
            }
        }
        free(xq); free(xqd); free(bias); free(x); free(m); free(wv); free(wc); free(wf); free(wa); free(wi);
    }
    return bad;
}
