/*
 * Plain FP64 CPU oracle of the triangular Yee-like leap-frog solver (arXiv:1812.01448).
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the CPU
 * baseline of the benchmark; never by the library.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

enum {
    ORC_OK = 0,
    ORC_EINVAL = -1,
    ORC_ENOTDELAUNAY = -2,
    ORC_EDEGENERATE = -3,
    ORC_ENONMANIFOLD = -4,
    ORC_EPERIODIC = -5,
    ORC_ENOTCONVERGED = -9,
};

enum { ORC_ORDER_NONE = 0, ORC_ORDER_RANDOM = 1, ORC_ORDER_MORTON = 2, ORC_ORDER_RCM = 3 };

typedef struct orc_mesh orc_mesh;

typedef struct {
    double dt;
    const double *gamma;     /* per-edge coefficient scale, NULL = 1 */
    const double *wp2;       /* per-edge plasma frequency squared, NULL = vacuum */
    double nu;               /* collision frequency */
    int64_t n_src;           /* soft source: edges, weights, waveform */
    const int32_t *src_edge;
    const double *src_w;
    double src_omega, src_cycles;
} orc_params;

uint64_t orc_splitmix64(uint64_t x);
/* threads of the per-cell loops (results do not depend on it) */
void orc_set_threads(int n);
int orc_get_threads(void);
uint64_t orc_morton(uint32_t qx, uint32_t qz);

orc_mesh *orc_mesh_build(const double *xy, int64_t nv, const int32_t *tri, int64_t nt,
                         int periodic, double Lx, double Ly, double dual_tol, int *status);
void orc_mesh_free(orc_mesh *m);
void orc_mesh_sizes(const orc_mesh *m, int64_t out[4]);
void orc_mesh_topology(const orc_mesh *m, int32_t *tri, int32_t *edge, int32_t *R, int32_t *L,
                       int32_t *A, int8_t *s);
void orc_mesh_geometry(const orc_mesh *m, double *elen, double *hR, double *hL, double *d,
                       double *S, double *O, double *C, double *evec);
void orc_node_boundary(const orc_mesh *m, uint8_t *out);

void orc_apply_LB(const orc_mesh *m, const double *gamma, const double *B, double *out);
void orc_apply_LE(const orc_mesh *m, const double *gamma, const double *E, double *out);
int orc_step(const orc_mesh *m, const orc_params *p, int64_t n0, int64_t nsteps,
             double *E, double *B, double *J, double *Q, double *B_prev);
double orc_energy(const orc_mesh *m, const double *E, const double *Bold, const double *Bnew);
void orc_div(const orc_mesh *m, const double *E, double *out);
int orc_power(const orc_mesh *m, const double *gamma, int64_t max_iter, double rtol,
              uint64_t seed, double *lambda_out, int64_t *iters_out);
int orc_order(const orc_mesh *m, int kind, uint64_t seed, int32_t *perm_t, int32_t *perm_e);

#endif
