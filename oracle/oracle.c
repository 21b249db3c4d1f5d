/*
 * Plain FP64 CPU oracle of the leap-frog Maxwell solver on triangular Yee-like meshes
 * (Fadeev, "Numerical simulation of 2D electrodynamic problems with unstructured
 * triangular meshes", arXiv:1812.01448).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code with the library.
 *
 * Every routine is a scalar loop in the order the paper (or the reading noted beside it)
 * states.  Build with -O2 -ffp-contract=off so that no multiply-add is fused.
 *
 * Threads: the per-cell loops of the stepper (each cell's new value depends only on the
 * old values of its neighbours) are split over OpenMP threads; every cell's arithmetic and
 * its order are the same as in one thread, so the result does not depend on the thread
 * count.  The nodal charge is a gather per node over its edges in ascending edge order,
 * which is the order a serial scatter over the edges would add them in.  Reductions
 * (energies, inner products) stay serial.
 *
 * Conventions:
 *  - coordinates (x1, x2) = (x, z); normal n = x1 x x2; B is the normal component;
 *  - triangles are made counter-clockwise by swapping v1 and v2 when needed;
 *  - an edge joins node lo < hi and its vector e points lo -> hi (any direction is
 *    allowed, Fig. 2); canonical edge id = rank of (lo, hi) in lexicographic order;
 *  - R(i) is the triangle whose counter-clockwise boundary runs lo -> hi along edge i,
 *    L(i) the other one (-1 when absent: an outer edge of a closed resonator);
 *  - A(j,q) is the edge from local vertex q to q+1 of triangle j, and
 *    s(j,q) = +1 if j = R(A(j,q)), else -1 (the sign of eq. 4, read topologically);
 *  - dual length d_i = hR_i + hL_i, signed half lengths from the edge midpoint to the
 *    two circumcentres along the left normal of e_i (|O_R O_L| of eq. 3 on a Delaunay mesh).
 *
 * The source waveform g(t) (`waveform`) is a reading (the paper does not specify its
 * source); its values are pinned at hand-evaluated times through the first step of a source
 * edge, besides the linearity of the response and the Gauss law with the source charge.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#include "oracle.h"

void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------- */
/* small helpers                                                              */
/* ------------------------------------------------------------------------- */

/* minimum-image difference on a periodic axis of length Lp (no change when closed) */
static double min_image(double delta, double Lp, int periodic)
{
    if (!periodic) return delta;
    return delta - Lp * nearbyint(delta / Lp);
}

/* splitmix64 (Steele, Lea and Flood, 2014): the published 64-bit mixing generator */
uint64_t orc_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------- */
/* mesh object                                                                */
/* ------------------------------------------------------------------------- */

struct orc_mesh {
    int64_t nv, nt, ne, nb;
    int periodic;
    double Lx, Ly;
    double *xy;          /* [nv][2] */
    int32_t *tri;        /* [nt][3], counter-clockwise */
    int32_t *edge;       /* [ne][2] = (lo, hi) */
    int32_t *R, *L;      /* [ne] */
    int32_t *A;          /* [nt][3] */
    int8_t *s;           /* [nt][3] */
    double *ex, *ez;     /* [ne] edge vector e = x_hi - x_lo (unwrapped) */
    double *elen;        /* [ne] |e| */
    double *hR, *hL, *d; /* [ne] half dual lengths and dual length */
    double *S;           /* [nt] area */
    double *O;           /* [nt][2] circumcentre (vertex 0 + local offset, not wrapped) */
    double *C;           /* [ne][2] edge midpoint x_lo + e/2 */
    uint8_t *node_bnd;   /* [nv] 1 if the node lies on an outer edge */
    int64_t *node_off;   /* [nv + 1] edges of node k: node_edge[node_off[k] .. node_off[k+1]) */
    int32_t *node_edge;  /* [2 ne] in ascending edge id */
};

typedef struct { int32_t lo, hi, t, q; int dir; } halfedge;

static int cmp_halfedge(const void *pa, const void *pb)
{
    const halfedge *a = (const halfedge *)pa, *b = (const halfedge *)pb;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    if (a->t != b->t) return a->t < b->t ? -1 : 1;
    return a->q < b->q ? -1 : (a->q > b->q);
}

void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->xy); free(m->tri); free(m->edge); free(m->R); free(m->L); free(m->A);
    free(m->s); free(m->ex); free(m->ez); free(m->elen); free(m->hR); free(m->hL);
    free(m->d); free(m->S); free(m->O); free(m->C); free(m->node_bnd);
    free(m->node_off); free(m->node_edge);
    free(m);
}

/* Local vertex positions of triangle j in its own frame (origin at vertex 0). */
static void local_frame(const orc_mesh *m, int64_t j, double P[3][2])
{
    const int32_t *v = m->tri + 3 * j;
    double ax = m->xy[2 * v[0]], az = m->xy[2 * v[0] + 1];
    P[0][0] = 0.0; P[0][1] = 0.0;
    for (int q = 1; q < 3; ++q) {
        P[q][0] = min_image(m->xy[2 * v[q]] - ax, m->Lx, m->periodic);
        P[q][1] = min_image(m->xy[2 * v[q] + 1] - az, m->Ly, m->periodic);
    }
}

/* Circumcentre offset u of a triangle with vertices 0, b, c (Fig. 2: O_j). */
static void circumcentre(const double b[2], const double c[2], double u[2], double *area)
{
    double o = b[0] * c[1] - b[1] * c[0];
    double D = 2.0 * o;
    double b2 = b[0] * b[0] + b[1] * b[1];
    double c2 = c[0] * c[0] + c[1] * c[1];
    u[0] = (c[1] * b2 - b[1] * c2) / D;
    u[1] = (b[0] * c2 - c[0] * b2) / D;
    *area = o / 2.0;
}

orc_mesh *orc_mesh_build(const double *xy, int64_t nv, const int32_t *tri_in, int64_t nt,
                         int periodic, double Lx, double Ly, double dual_tol, int *status)
{
    *status = ORC_EINVAL;
    if (nv <= 0 || nt <= 0 || !(Lx > 0.0) || !(Ly > 0.0)) return NULL;
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    m->nv = nv; m->nt = nt; m->periodic = periodic; m->Lx = Lx; m->Ly = Ly;
    m->xy = (double *)malloc(sizeof(double) * 2 * nv);
    memcpy(m->xy, xy, sizeof(double) * 2 * nv);
    m->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
    for (int64_t k = 0; k < 3 * nt; ++k) {
        if (tri_in[k] < 0 || tri_in[k] >= nv) { orc_mesh_free(m); return NULL; }
        m->tri[k] = tri_in[k];
    }

    /* orientation: counter-clockwise by swapping v1 and v2 (degenerate -> error) */
    for (int64_t j = 0; j < nt; ++j) {
        double P[3][2];
        local_frame(m, j, P);
        double o = P[1][0] * P[2][1] - P[1][1] * P[2][0];
        if (fabs(o) <= 1e-14 * Lx * Ly) { *status = ORC_EDEGENERATE; orc_mesh_free(m); return NULL; }
        if (o < 0.0) {
            int32_t tmp = m->tri[3 * j + 1];
            m->tri[3 * j + 1] = m->tri[3 * j + 2];
            m->tri[3 * j + 2] = tmp;
        }
    }

    /* edges: sort the 3*nt directed sides by their undirected key */
    halfedge *he = (halfedge *)malloc(sizeof(halfedge) * 3 * nt);
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q) {
            int32_t a = m->tri[3 * j + q], b = m->tri[3 * j + (q + 1) % 3];
            halfedge *h = &he[3 * j + q];
            h->lo = a < b ? a : b; h->hi = a < b ? b : a;
            h->t = (int32_t)j; h->q = q; h->dir = a < b ? +1 : -1;
        }
    qsort(he, (size_t)(3 * nt), sizeof(halfedge), cmp_halfedge);

    int64_t ne = 0;
    for (int64_t k = 0; k < 3 * nt; ++k)
        if (k == 0 || he[k].lo != he[k - 1].lo || he[k].hi != he[k - 1].hi) ++ne;
    m->ne = ne;
    m->edge = (int32_t *)malloc(sizeof(int32_t) * 2 * ne);
    m->R = (int32_t *)malloc(sizeof(int32_t) * ne);
    m->L = (int32_t *)malloc(sizeof(int32_t) * ne);
    m->A = (int32_t *)malloc(sizeof(int32_t) * 3 * nt);
    m->s = (int8_t *)malloc(sizeof(int8_t) * 3 * nt);

    int64_t id = -1, nb = 0;
    for (int64_t k = 0; k < 3 * nt;) {
        int64_t g = k;
        while (g < 3 * nt && he[g].lo == he[k].lo && he[g].hi == he[k].hi) ++g;
        ++id;
        m->edge[2 * id] = he[k].lo;
        m->edge[2 * id + 1] = he[k].hi;
        m->R[id] = -1; m->L[id] = -1;
        int64_t cnt = g - k;
        if (cnt > 2) { *status = ORC_ENONMANIFOLD; free(he); orc_mesh_free(m); return NULL; }
        for (int64_t r = k; r < g; ++r) {
            if (he[r].dir > 0) {
                if (m->R[id] >= 0) { *status = ORC_ENONMANIFOLD; free(he); orc_mesh_free(m); return NULL; }
                m->R[id] = he[r].t;
            } else {
                if (m->L[id] >= 0) { *status = ORC_ENONMANIFOLD; free(he); orc_mesh_free(m); return NULL; }
                m->L[id] = he[r].t;
            }
            m->A[3 * he[r].t + he[r].q] = (int32_t)id;
        }
        if (cnt == 1) {
            if (periodic) { *status = ORC_EPERIODIC; free(he); orc_mesh_free(m); return NULL; }
            ++nb;
        }
        k = g;
    }
    free(he);
    m->nb = nb;
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q)
            m->s[3 * j + q] = (int8_t)(m->R[m->A[3 * j + q]] == j ? +1 : -1);

    /* geometry (eqs. 3, 4, 7): per-triangle frames, circumcentres, half dual lengths */
    m->ex = (double *)malloc(sizeof(double) * ne);
    m->ez = (double *)malloc(sizeof(double) * ne);
    m->elen = (double *)malloc(sizeof(double) * ne);
    m->hR = (double *)calloc((size_t)ne, sizeof(double));
    m->hL = (double *)calloc((size_t)ne, sizeof(double));
    m->d = (double *)malloc(sizeof(double) * ne);
    m->S = (double *)malloc(sizeof(double) * nt);
    m->O = (double *)malloc(sizeof(double) * 2 * nt);
    m->C = (double *)malloc(sizeof(double) * 2 * ne);
    m->node_bnd = (uint8_t *)calloc((size_t)nv, 1);

    for (int64_t i = 0; i < ne; ++i) {
        int32_t lo = m->edge[2 * i], hi = m->edge[2 * i + 1];
        m->ex[i] = min_image(m->xy[2 * hi] - m->xy[2 * lo], Lx, periodic);
        m->ez[i] = min_image(m->xy[2 * hi + 1] - m->xy[2 * lo + 1], Ly, periodic);
        m->elen[i] = hypot(m->ex[i], m->ez[i]);
        m->C[2 * i] = m->xy[2 * lo] + m->ex[i] / 2.0;
        m->C[2 * i + 1] = m->xy[2 * lo + 1] + m->ez[i] / 2.0;
        if (m->R[i] < 0 || m->L[i] < 0) { m->node_bnd[lo] = 1; m->node_bnd[hi] = 1; }
    }

    for (int64_t j = 0; j < nt; ++j) {
        double P[3][2], u[2], area;
        local_frame(m, j, P);
        circumcentre(P[1], P[2], u, &area);
        m->S[j] = area;
        const int32_t *v = m->tri + 3 * j;
        m->O[2 * j] = m->xy[2 * v[0]] + u[0];
        m->O[2 * j + 1] = m->xy[2 * v[0] + 1] + u[1];
        for (int q = 0; q < 3; ++q) {
            int32_t i = m->A[3 * j + q];
            double tx = m->ex[i] / m->elen[i], tz = m->ez[i] / m->elen[i];
            double nx = -tz, nz = tx;            /* left normal of e_i */
            const double *plo, *phi;
            if (m->s[3 * j + q] > 0) { plo = P[q]; phi = P[(q + 1) % 3]; }
            else                     { plo = P[(q + 1) % 3]; phi = P[q]; }
            double cx = (plo[0] + phi[0]) / 2.0, cz = (plo[1] + phi[1]) / 2.0;
            if (m->s[3 * j + q] > 0) m->hR[i] = (u[0] - cx) * nx + (u[1] - cz) * nz;
            else                     m->hL[i] = (cx - u[0]) * nx + (cz - u[1]) * nz;
        }
    }
    for (int64_t i = 0; i < ne; ++i) {
        m->d[i] = m->hR[i] + m->hL[i];
        if (m->R[i] >= 0 && m->L[i] >= 0 && !(m->d[i] > dual_tol * m->elen[i])) {
            *status = ORC_ENOTDELAUNAY; orc_mesh_free(m); return NULL;
        }
    }

    /* node -> edge incidence lists, each in ascending edge id (for the nodal charge) */
    m->node_off = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
    m->node_edge = (int32_t *)malloc(sizeof(int32_t) * 2 * ne);
    for (int64_t i = 0; i < ne; ++i) {
        ++m->node_off[m->edge[2 * i] + 1];
        ++m->node_off[m->edge[2 * i + 1] + 1];
    }
    for (int64_t v = 0; v < nv; ++v) m->node_off[v + 1] += m->node_off[v];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * nv);
        memcpy(fill, m->node_off, sizeof(int64_t) * nv);
        for (int64_t i = 0; i < ne; ++i) {
            m->node_edge[fill[m->edge[2 * i]]++] = (int32_t)i;
            m->node_edge[fill[m->edge[2 * i + 1]]++] = (int32_t)i;
        }
        free(fill);
    }
    *status = ORC_OK;
    return m;
}

void orc_mesh_sizes(const orc_mesh *m, int64_t out[4])
{
    out[0] = m->nv; out[1] = m->ne; out[2] = m->nt; out[3] = m->nb;
}

void orc_mesh_topology(const orc_mesh *m, int32_t *tri, int32_t *edge, int32_t *R, int32_t *L,
                       int32_t *A, int8_t *s)
{
    if (tri) memcpy(tri, m->tri, sizeof(int32_t) * 3 * m->nt);
    if (edge) memcpy(edge, m->edge, sizeof(int32_t) * 2 * m->ne);
    if (R) memcpy(R, m->R, sizeof(int32_t) * m->ne);
    if (L) memcpy(L, m->L, sizeof(int32_t) * m->ne);
    if (A) memcpy(A, m->A, sizeof(int32_t) * 3 * m->nt);
    if (s) memcpy(s, m->s, sizeof(int8_t) * 3 * m->nt);
}

void orc_mesh_geometry(const orc_mesh *m, double *elen, double *hR, double *hL, double *d,
                       double *S, double *O, double *C, double *evec)
{
    int64_t ne = m->ne, nt = m->nt;
    if (elen) memcpy(elen, m->elen, sizeof(double) * ne);
    if (hR) memcpy(hR, m->hR, sizeof(double) * ne);
    if (hL) memcpy(hL, m->hL, sizeof(double) * ne);
    if (d) memcpy(d, m->d, sizeof(double) * ne);
    if (S) memcpy(S, m->S, sizeof(double) * nt);
    if (O) memcpy(O, m->O, sizeof(double) * 2 * nt);
    if (C) memcpy(C, m->C, sizeof(double) * 2 * ne);
    if (evec)
        for (int64_t i = 0; i < ne; ++i) { evec[2 * i] = m->ex[i]; evec[2 * i + 1] = m->ez[i]; }
}

void orc_node_boundary(const orc_mesh *m, uint8_t *out)
{
    memcpy(out, m->node_bnd, (size_t)m->nv);
}

/* ------------------------------------------------------------------------- */
/* discrete curl operators (eq. 3 and eq. 4), optional per-edge scale gamma     */
/* ------------------------------------------------------------------------- */

static int interior(const orc_mesh *m, int64_t i) { return m->R[i] >= 0 && m->L[i] >= 0; }

/* (L_B B)_i = gamma_i (B_R - B_L) / d_i on interior edges, 0 on outer edges (eq. 3) */
void orc_apply_LB(const orc_mesh *m, const double *gamma, const double *B, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m->ne; ++i) {
        if (!interior(m, i)) { out[i] = 0.0; continue; }
        double g = gamma ? gamma[i] : 1.0;
        out[i] = g * (B[m->R[i]] - B[m->L[i]]) / m->d[i];
    }
}

/* (L_E E)_j = -(1/S_j) sum_q s(j,q) gamma |e| E over the three edges, q = 0, 1, 2 (eq. 4) */
void orc_apply_LE(const orc_mesh *m, const double *gamma, const double *E, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m->nt; ++j) {
        double acc = 0.0;
        for (int q = 0; q < 3; ++q) {
            int32_t i = m->A[3 * j + q];
            double g = gamma ? gamma[i] : 1.0;
            acc += (double)m->s[3 * j + q] * g * m->elen[i] * E[i];
        }
        out[j] = -acc / m->S[j];
    }
}

/* ------------------------------------------------------------------------- */
/* leap-frog stepping with Drude current, nodal charge and soft source          */
/* ------------------------------------------------------------------------- */

/* soft-source envelope g(t) = sin(omega t) sin^2(pi t / T), T = cycles 2 pi / omega, zero
   outside [0, T) (a reading: Fig. 3's source is unspecified) */
static double waveform(double t, double omega, double cycles)
{
    double T = cycles * 2.0 * M_PI / omega;
    if (!(t >= 0.0 && t < T)) return 0.0;
    double s = sin(M_PI * t / T);
    return sin(omega * t) * s * s;
}

/*
 * One call advances nsteps leap-frog steps starting at global step index n0.
 * On entry: E = E^n0, B = B^(n0+1/2), J = j^(n0-1/2), Q = Q^n0.
 * Step n -> n+1 (eqs. 3-6 with the physical Drude sign and a Crank-Nicolson collision term):
 *   j^(n+1/2) = [(1 - nu dt/2) j^(n-1/2) + dt wp2 E^n] / (1 + nu dt/2)   (plasma edges)
 *   E^(n+1)   = E^n + dt [ (L_B B^(n+1/2)) - j^(n+1/2) - Jsrc(t^(n+1/2)) ]  (interior edges)
 *   Q^(n+1)   = Q^n - dt sum_i sigma(k,i) d_i (j + Jsrc)_i                  (interior nodes)
 *   B^(n+3/2) = B^(n+1/2) + dt (L_E E^(n+1))
 * B_prev (optional) receives B^(n0+nsteps-1/2) for the leap-frog energy.
 */
int orc_step(const orc_mesh *m, const orc_params *p, int64_t n0, int64_t nsteps,
             double *E, double *B, double *J, double *Q, double *B_prev)
{
    int64_t ne = m->ne, nt = m->nt, nv = m->nv;
    double dt = p->dt;
    int media = p->wp2 != NULL;
    int source = p->n_src > 0;
    if ((media && !J) || ((media || source) && !Q)) return ORC_EINVAL;
    double *LB = (double *)malloc(sizeof(double) * ne);
    double *LE = (double *)malloc(sizeof(double) * nt);
    double *Js = (double *)calloc((size_t)ne, sizeof(double));
    for (int64_t k = 0; k < nsteps; ++k) {
        int64_t n = n0 + k;
        double th = ((double)n + 0.5) * dt;
        if (media) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < ne; ++i)
                if (p->wp2[i] > 0.0)
                    J[i] = ((1.0 - p->nu * dt / 2.0) * J[i] + dt * p->wp2[i] * E[i])
                           / (1.0 + p->nu * dt / 2.0);
        }
        if (source) {
            double g = waveform(th, p->src_omega, p->src_cycles);
            memset(Js, 0, sizeof(double) * ne);
            for (int64_t r = 0; r < p->n_src; ++r) Js[p->src_edge[r]] += p->src_w[r] * g;
        }
        orc_apply_LB(m, p->gamma, B, LB);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < ne; ++i) {
            if (!interior(m, i)) continue;
            double rhs = LB[i];
            if (media) rhs -= J[i];
            if (source) rhs -= Js[i];
            E[i] = E[i] + dt * rhs;
        }
        if (media || source) {
            /* flux of (j + Jsrc) out of node v: + d_i cur_i where e_i leaves v (v = lo),
               - d_i cur_i where it enters (v = hi), over v's edges in ascending id */
#pragma omp parallel for schedule(static)
            for (int64_t v = 0; v < nv; ++v) {
                if (m->node_bnd[v]) continue;
                double flux = 0.0;
                for (int64_t r = m->node_off[v]; r < m->node_off[v + 1]; ++r) {
                    int64_t i = m->node_edge[r];
                    double cur = (media ? J[i] : 0.0) + (source ? Js[i] : 0.0);
                    if (cur == 0.0) continue;
                    if (m->edge[2 * i] == v) flux += m->d[i] * cur;
                    else                     flux -= m->d[i] * cur;
                }
                Q[v] = Q[v] - dt * flux;
            }
        }
        orc_apply_LE(m, p->gamma, E, LE);
        if (B_prev && k == nsteps - 1) memcpy(B_prev, B, sizeof(double) * nt);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nt; ++j) B[j] = B[j] + dt * LE[j];
    }
    free(LB); free(LE); free(Js);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* diagnostics (eqs. 7-10; div E as the flux through the Voronoi cell, Section 1)  */
/* ------------------------------------------------------------------------- */

/* W_h = sum_i w_i E_i^2 + sum_j S_j Bold_j Bnew_j, w_i = d_i |e_i| (metric (7)); with
   Bold = Bnew this is the instantaneous energy of eq. 8 with signed dual lengths. */
double orc_energy(const orc_mesh *m, const double *E, const double *Bold, const double *Bnew)
{
    double we = 0.0, wb = 0.0;
    for (int64_t i = 0; i < m->ne; ++i)
        if (interior(m, i)) we += m->d[i] * m->elen[i] * E[i] * E[i];
    for (int64_t j = 0; j < m->nt; ++j) wb += m->S[j] * Bold[j] * Bnew[j];
    return we + wb;
}

/* (DE)_k = sum_i sigma(k,i) d_i E_i, sigma = +1 when e_i points away from node k */
void orc_div(const orc_mesh *m, const double *E, double *out)
{
    memset(out, 0, sizeof(double) * m->nv);
    for (int64_t i = 0; i < m->ne; ++i) {
        out[m->edge[2 * i]] += m->d[i] * E[i];
        out[m->edge[2 * i + 1]] -= m->d[i] * E[i];
    }
}

/* ------------------------------------------------------------------------- */
/* largest eigenvalue of K = -L_E L_B by normalised iteration (Section 2), S-weighted */
/* ------------------------------------------------------------------------- */

static void apply_K(const orc_mesh *m, const double *gamma, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m->nt; ++j) {
        double acc = 0.0;
        for (int q = 0; q < 3; ++q) {
            int32_t i = m->A[3 * j + q];
            if (!interior(m, i)) continue;
            double g = gamma ? gamma[i] : 1.0;
            double wt = g * g * m->elen[i] / m->d[i];
            int32_t other = m->R[i] == j ? m->L[i] : m->R[i];
            acc += wt * (x[j] - x[other]);
        }
        y[j] = acc / m->S[j];
    }
}

int orc_power(const orc_mesh *m, const double *gamma, int64_t max_iter, double rtol,
              uint64_t seed, double *lambda_out, int64_t *iters_out)
{
    int64_t nt = m->nt;
    double *x = (double *)malloc(sizeof(double) * nt);
    double *y = (double *)malloc(sizeof(double) * nt);
    for (int64_t j = 0; j < nt; ++j) {
        uint64_t z = orc_splitmix64(seed + (uint64_t)j);
        double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        x[j] = 2.0 * u - 1.0;
    }
    double lam = 0.0, lam_prev = 0.0;
    int64_t it;
    int converged = 0;
    for (it = 1; it <= max_iter; ++it) {
        apply_K(m, gamma, x, y);
        double xy = 0.0, xx = 0.0, yy = 0.0;
        for (int64_t j = 0; j < nt; ++j) {
            xy += m->S[j] * x[j] * y[j];
            xx += m->S[j] * x[j] * x[j];
            yy += m->S[j] * y[j] * y[j];
        }
        lam = xy / xx;
        double ny = sqrt(yy);
        for (int64_t j = 0; j < nt; ++j) x[j] = y[j] / ny;
        if (it > 1 && fabs(lam - lam_prev) <= rtol * lam) { converged = 1; break; }
        lam_prev = lam;
    }
    free(x); free(y);
    *lambda_out = lam;
    *iters_out = converged ? it : max_iter;
    return converged ? ORC_OK : ORC_ENOTCONVERGED;
}

/* ------------------------------------------------------------------------- */
/* locality orderings (new -> canonical maps)                                  */
/* ------------------------------------------------------------------------- */

typedef struct { uint64_t key; int64_t id; } keyed;

static int cmp_keyed(const void *pa, const void *pb)
{
    const keyed *a = (const keyed *)pa, *b = (const keyed *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

static void sort_by_keys(keyed *k, int64_t n, int32_t *perm)
{
    qsort(k, (size_t)n, sizeof(keyed), cmp_keyed);
    for (int64_t r = 0; r < n; ++r) perm[r] = (int32_t)k[r].id;
}

static double wrap(double v, double Lp) { return v - Lp * floor(v / Lp); }

static uint32_t quantise16(double c, double Lp)
{
    double q = floor(c / Lp * 65536.0);
    if (q < 0.0) q = 0.0;
    if (q > 65535.0) q = 65535.0;
    return (uint32_t)q;
}

/* bit-interleave: bit b of qx goes to bit 2b, bit b of qz to bit 2b+1 */
uint64_t orc_morton(uint32_t qx, uint32_t qz)
{
    uint64_t key = 0;
    for (int b = 0; b < 16; ++b) {
        key |= (uint64_t)((qx >> b) & 1u) << (2 * b);
        key |= (uint64_t)((qz >> b) & 1u) << (2 * b + 1);
    }
    return key;
}

static int degree(const orc_mesh *m, int64_t j)
{
    int deg = 0;
    for (int q = 0; q < 3; ++q) deg += interior(m, m->A[3 * j + q]);
    return deg;
}

static int64_t neighbour(const orc_mesh *m, int64_t j, int q)
{
    int32_t i = m->A[3 * j + q];
    if (!interior(m, i)) return -1;
    return m->R[i] == j ? m->L[i] : m->R[i];
}

/* breadth-first levels from r inside its component; returns the eccentricity and fills
   `last` with the argmin (degree, id) of the deepest level */
static int64_t bfs_levels(const orc_mesh *m, int64_t r, int64_t *level, int64_t *queue,
                          int64_t *last)
{
    int64_t head = 0, tail = 0;
    level[r] = 0;
    queue[tail++] = r;
    while (head < tail) {
        int64_t j = queue[head++];
        for (int q = 0; q < 3; ++q) {
            int64_t k = neighbour(m, j, q);
            if (k >= 0 && level[k] < 0) { level[k] = level[j] + 1; queue[tail++] = k; }
        }
    }
    int64_t ecc = level[queue[tail - 1]];
    int64_t best = -1;
    for (int64_t t = 0; t < tail; ++t) {
        int64_t j = queue[t];
        if (level[j] != ecc) continue;
        if (best < 0 || degree(m, j) < degree(m, best) ||
            (degree(m, j) == degree(m, best) && j < best)) best = j;
    }
    for (int64_t t = 0; t < tail; ++t) level[queue[t]] = -1;  /* reset for the next BFS */
    *last = best;
    return ecc;
}

typedef struct { int deg; int64_t id; } degid;

static int cmp_degid(const void *pa, const void *pb)
{
    const degid *a = (const degid *)pa, *b = (const degid *)pb;
    if (a->deg != b->deg) return a->deg < b->deg ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id);
}

/* reverse Cuthill-McKee on the triangle adjacency (triangles sharing an interior edge),
   starting each component from a George-Liu pseudo-peripheral triangle */
static void order_rcm(const orc_mesh *m, int32_t *perm_t)
{
    int64_t nt = m->nt;
    int64_t *level = (int64_t *)malloc(sizeof(int64_t) * nt);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * nt);
    uint8_t *seen = (uint8_t *)calloc((size_t)nt, 1);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * nt);
    for (int64_t j = 0; j < nt; ++j) level[j] = -1;
    int64_t count = 0;
    while (count < nt) {
        int64_t r = -1;
        for (int64_t j = 0; j < nt; ++j)
            if (!seen[j] && (r < 0 || degree(m, j) < degree(m, r))) r = j;
        int64_t cand;
        int64_t ecc = bfs_levels(m, r, level, queue, &cand);
        for (;;) {
            int64_t cand2;
            int64_t ecc2 = bfs_levels(m, cand, level, queue, &cand2);
            if (ecc2 > ecc) { r = cand; ecc = ecc2; cand = cand2; }
            else break;
        }
        int64_t head = count;
        order[count++] = r;
        seen[r] = 1;
        while (head < count) {
            int64_t j = order[head++];
            degid nb[3];
            int cnt = 0;
            for (int q = 0; q < 3; ++q) {
                int64_t k = neighbour(m, j, q);
                if (k >= 0 && !seen[k]) {
                    int dup = 0;
                    for (int c = 0; c < cnt; ++c) dup |= nb[c].id == k;
                    if (!dup) { nb[cnt].deg = degree(m, k); nb[cnt].id = k; ++cnt; }
                }
            }
            qsort(nb, (size_t)cnt, sizeof(degid), cmp_degid);
            for (int c = 0; c < cnt; ++c) { seen[nb[c].id] = 1; order[count++] = nb[c].id; }
        }
    }
    for (int64_t r = 0; r < nt; ++r) perm_t[r] = (int32_t)order[nt - 1 - r];
    free(level); free(queue); free(seen); free(order);
}

/* edges in order of first appearance over (new triangle order, q = 0, 1, 2) */
static void edges_first_appearance(const orc_mesh *m, const int32_t *perm_t, int32_t *perm_e)
{
    uint8_t *seen = (uint8_t *)calloc((size_t)m->ne, 1);
    int64_t c = 0;
    for (int64_t r = 0; r < m->nt; ++r)
        for (int q = 0; q < 3; ++q) {
            int32_t i = m->A[3 * perm_t[r] + q];
            if (!seen[i]) { seen[i] = 1; perm_e[c++] = i; }
        }
    free(seen);
}

int orc_order(const orc_mesh *m, int kind, uint64_t seed, int32_t *perm_t, int32_t *perm_e)
{
    int64_t nt = m->nt, ne = m->ne;
    if (kind == ORC_ORDER_NONE) {
        for (int64_t j = 0; j < nt; ++j) perm_t[j] = (int32_t)j;
        for (int64_t i = 0; i < ne; ++i) perm_e[i] = (int32_t)i;
        return ORC_OK;
    }
    if (kind == ORC_ORDER_RANDOM) {
        keyed *k = (keyed *)malloc(sizeof(keyed) * (nt > ne ? nt : ne));
        for (int64_t j = 0; j < nt; ++j) { k[j].key = orc_splitmix64(seed + (uint64_t)j); k[j].id = j; }
        sort_by_keys(k, nt, perm_t);
        for (int64_t i = 0; i < ne; ++i) {
            k[i].key = orc_splitmix64(seed + (uint64_t)nt + (uint64_t)i);
            k[i].id = i;
        }
        sort_by_keys(k, ne, perm_e);
        free(k);
        return ORC_OK;
    }
    if (kind == ORC_ORDER_MORTON) {
        keyed *k = (keyed *)malloc(sizeof(keyed) * nt);
        for (int64_t j = 0; j < nt; ++j) {
            const int32_t *v = m->tri + 3 * j;
            double c[2];
            for (int ax = 0; ax < 2; ++ax) {
                double Lp = ax == 0 ? m->Lx : m->Ly;
                double xa = m->xy[2 * v[0] + ax], xb = m->xy[2 * v[1] + ax], xc = m->xy[2 * v[2] + ax];
                if (m->periodic) {
                    double ub = min_image(xb - xa, Lp, 1), uc = min_image(xc - xa, Lp, 1);
                    c[ax] = wrap(xa + (ub + uc) / 3.0, Lp);
                } else {
                    c[ax] = ((xa + xb) + xc) / 3.0;
                }
            }
            k[j].key = orc_morton(quantise16(c[0], m->Lx), quantise16(c[1], m->Ly));
            k[j].id = j;
        }
        sort_by_keys(k, nt, perm_t);
        free(k);
        edges_first_appearance(m, perm_t, perm_e);
        return ORC_OK;
    }
    if (kind == ORC_ORDER_RCM) {
        order_rcm(m, perm_t);
        edges_first_appearance(m, perm_t, perm_e);
        return ORC_OK;
    }
    return ORC_EINVAL;
}
