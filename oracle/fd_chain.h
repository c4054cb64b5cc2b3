/*
 * fd_chain.h -- the oracle's view of one chain inside packed per-link arrays.
 * TEST INFRASTRUCTURE ONLY (see fd_oracle.c).
 */
#ifndef FD_ORACLE_CHAIN_H
#define FD_ORACLE_CHAIN_H
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* A robot: n links; link i hangs from link parent[i] (< i) of the same robot, or
 * from the base when parent[i] is -1. parent == NULL: a serial chain (i - 1). */
typedef struct {
    int n;
    const double *axis, *home_rot, *offset, *mass, *com, *inertia;
    const int32_t *parent;
    double g[3];
} chain_t;

typedef struct {
    const double *axis, *home_rot, *offset, *mass, *com, *inertia, *gravity;
    const int32_t *parent;
} model_arrays_t;

static inline int parent_of(const chain_t *c, int i) { return c->parent ? c->parent[i] : i - 1; }

static inline chain_t chain_at(const model_arrays_t *ma, int64_t start, int n) {
    chain_t c;
    c.n = n;
    c.axis = ma->axis + 3 * start;
    c.home_rot = ma->home_rot + 9 * start;
    c.offset = ma->offset + 3 * start;
    c.mass = ma->mass + start;
    c.com = ma->com + 3 * start;
    c.inertia = ma->inertia + 6 * start;
    c.parent = ma->parent ? ma->parent + start : NULL;
    for (int a = 0; a < 3; ++a) c.g[a] = ma->gravity[a];
    return c;
}

static inline void set_threads(int nthreads) {
#ifdef _OPENMP
    omp_set_num_threads(nthreads > 0 ? nthreads : omp_get_num_procs());
#else
    (void)nthreads;
#endif
}


#define MODEL_ARGS                                                                          \
    const double *axis, const double *home_rot, const double *offset, const double *mass,   \
        const double *com, const double *inertia, const double *gravity, const int32_t *parent
#define MODEL_INIT model_arrays_t ma = {axis, home_rot, offset, mass, com, inertia, gravity, parent}
#define MSTART(b) (model_start ? model_start[b] : offsets[b])

#endif
