/*
 * tyee — leap-frog Maxwell solver on unstructured triangular Yee-like meshes, for AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Fadeev, "Numerical simulation of 2D electrodynamic problems with unstructured
 * triangular meshes", arXiv:1812.01448.  Section numbers and equation numbers below refer
 * to that paper.
 *
 * Placement (Section 1, Fig. 1 and Fig. 2): E_i is the projection of the electric field on
 * mesh edge i at its midpoint C_i; the single magnetic component B_j sits at the
 * circumcentre O_j of triangle j; plasma currents j_i share the edges with E; charge sits on
 * nodes.  The plane carries coordinates (x1, x2); B is the component along x1 x x2.
 *
 * Numbering (canonical, independent of any reordering):
 *   - triangle j = row j of the triangle array handed to tyee_mesh_create; its vertices are
 *     made counter-clockwise by swapping v1 and v2 when needed;
 *   - edge i = rank of its node pair (lo < hi) in lexicographic order; its vector e_i
 *     points lo -> hi (the paper allows any direction, Fig. 2);
 *   - R(i) is the triangle whose counter-clockwise boundary runs lo -> hi along edge i, L(i)
 *     the other (-1 on an outer edge of a closed resonator);
 *   - A(j,q) is the edge from local vertex q to q+1 of triangle j; s(j,q) = +1 when
 *     j = R(A(j,q)), else -1 (the sign of eq. 4 read from the mesh topology).
 * Geometry is computed in FP64 in each triangle's own frame: area S_j, circumcentre O_j,
 * signed half dual lengths hR_i = (O_R - C_i).n_i and hL_i = (C_i - O_L).n_i with n_i the
 * left normal of e_i, and dual length d_i = hR_i + hL_i (|O_R O_L| of eq. 3 on a Delaunay
 * mesh).
 *
 * Time levels: E and Q at t = n dt; B and j at t = (n + 1/2) dt.  One step (eqs. 3-6):
 *   j  <- [(1 - nu dt/2) j + dt wp2 E] / (1 + nu dt/2)             (plasma edges, eq. 5)
 *   E  <- E + dt [ gamma (B_R - B_L)/d - j - Jsrc(t + dt/2) ]       (interior edges, eqs. 3, 6)
 *   Q  <- Q - dt sum_i sigma(k,i) d_i (j + Jsrc)_i                  (interior nodes)
 *   B  <- B - (dt/S_j) sum_q s(j,q) gamma |e| E                      (eq. 4)
 * with gamma = 1 for the plain method (a per-edge scale for the learned correction).
 * Outer edges of a closed resonator carry E = 0 and are never updated (eqs. 9-10).
 *
 * Conventions for every call:
 *   - return 0 (TYEE_OK) on success or a negative tyee_status; tyee_last_error() then holds a
 *     message for the calling thread.  No C++ exception crosses this interface.
 *   - input arrays are copied; output arrays are caller-owned; views are borrowed and stay
 *     valid until the owning handle is destroyed or reordered.
 *   - a handle is not thread-safe; one simulation uses one HIP stream.
 *   - destroy functions accept NULL.
 */
#ifndef TYEE_H
#define TYEE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TYEE_OK = 0,
    TYEE_EINVAL = -1,        /* bad argument, size or state */
    TYEE_ENOTDELAUNAY = -2,  /* an interior edge has d_i <= dual_tol * |e_i| */
    TYEE_EDEGENERATE = -3,   /* a triangle with |2 S| <= 1e-14 Lx Ly; a tetrahedron with no volume */
    TYEE_ENONMANIFOLD = -4,  /* an edge in more than two triangles, or twice in one direction; a
                                face in more than two tetrahedra, or two on one of its sides */
    TYEE_EPERIODIC = -5,     /* periodic mesh with an edge that has only one triangle */
    TYEE_ENOMEM = -6,        /* host or device allocation failed */
    TYEE_EDEVICE = -7,       /* a HIP runtime call failed */
    TYEE_EUNSTABLE = -8,     /* non-finite field detected */
    TYEE_ENOTCONVERGED = -9  /* an iteration hit its limit (power iteration, modes) */
} tyee_status;

typedef enum { TYEE_PEC_BOX = 0, TYEE_PERIODIC = 1 } tyee_domain_kind;

/* kind: closed resonator (outer edges E = 0, eqs. 9-10) or periodic square (a torus).
   Lx, Ly: periods of a torus (positions are taken modulo them and differences by minimum
   image); for a box they only set the degeneracy scale Lx*Ly.  dual_tol: creation fails when
   an interior edge has d_i <= dual_tol * |e_i| (0 = require a strictly positive dual). */
typedef struct {
    int32_t kind;
    double Lx, Ly;
    double dual_tol;
} tyee_domain;

typedef enum { TYEE_ORDER_NONE = 0, TYEE_ORDER_RANDOM = 1, TYEE_ORDER_MORTON = 2,
               TYEE_ORDER_RCM = 3 } tyee_order;

typedef enum { TYEE_F32 = 0, TYEE_F64 = 1 } tyee_prec;

typedef enum { TYEE_FIELD_E = 0, TYEE_FIELD_B = 1, TYEE_FIELD_J = 2, TYEE_FIELD_Q = 3 } tyee_field;

typedef struct tyee_mesh tyee_mesh;
typedef struct tyee_sim tyee_sim;

typedef struct {
    int64_t n_nodes, n_edges, n_tris, n_boundary_edges;
    double min_dual_ratio, max_dual_ratio;  /* min / max of d_i/|e_i| over interior edges */
    double sum_area;                        /* sum_j S_j */
    double sum_dual_area;                   /* sum_i |e_i| d_i / 2 (equals sum_area) */
    int64_t n_obtuse;                       /* triangles whose circumcentre is outside */
} tyee_mesh_info;

/* Borrowed host views of a mesh, canonical numbering, FP64 geometry. */
typedef struct {
    const int32_t *tri;         /* [n_tris][3] counter-clockwise vertices */
    const int32_t *edge_nodes;  /* [n_edges][2] (lo, hi) */
    const int32_t *R, *L;       /* [n_edges] triangles left / right of e_i, -1 if none */
    const int32_t *A;           /* [n_tris][3] edges of each triangle */
    const int8_t *sgn;          /* [n_tris][3] s(j,q) */
    const double *elen;         /* [n_edges] |e_i| */
    const double *evec;         /* [n_edges][2] e_i = x_hi - x_lo (minimum image) */
    const double *hR, *hL, *d;  /* [n_edges] half dual lengths and dual length */
    const double *S;            /* [n_tris] areas */
    const double *O;            /* [n_tris][2] circumcentres (vertex 0 + local offset) */
    const double *C;            /* [n_edges][2] edge midpoints x_lo + e_i/2 */
    const int32_t *perm_t;      /* [n_tris]  device slot -> canonical triangle */
    const int32_t *perm_e;      /* [n_edges] device slot -> canonical edge */
} tyee_mesh_arrays;

/* ---------------------------------------------------------------- mesh ---- */

/* Build connectivity and geometry from a node cloud and triangles (Section 3 mesh
   creation; Fig. 2 quantities).  xy: [n_nodes][2] FP64 host; tri: [n_tris][3] int32 node
   indices, any winding.  Errors: TYEE_EINVAL, TYEE_EDEGENERATE, TYEE_ENONMANIFOLD,
   TYEE_EPERIODIC, TYEE_ENOTDELAUNAY, TYEE_ENOMEM.  *out receives a new handle. */
int tyee_mesh_create(const double *xy, int64_t n_nodes, const int32_t *tri, int64_t n_tris,
                     const tyee_domain *dom, tyee_mesh **out);

/* Choose the device numbering of triangles and edges for memory locality.  Always computed
   from the canonical numbering (idempotent).  NONE: identity.  RANDOM: triangles sorted by
   (splitmix64(seed + j), j), edges by (splitmix64(seed + n_tris + i), i).  MORTON: triangles
   by the 32-bit Z-order key of their vertex-average quantised to 16 bits per axis, ties by
   id.  RCM: reverse Cuthill-McKee on triangles sharing interior edges, each component
   started from a George-Liu pseudo-peripheral triangle, neighbours visited by (degree, id).
   MORTON and RCM number edges by first appearance over (new triangle order, q = 0, 1, 2).
   A simulation created afterwards uses this numbering on the device; results read back
   are always canonical. */
int tyee_mesh_reorder(tyee_mesh *mesh, int32_t kind, uint64_t seed);

/* Counts and the Section 3 quality measures of a mesh (out: caller-owned).  Errors: EINVAL. */
int tyee_mesh_query(const tyee_mesh *mesh, tyee_mesh_info *out);
/* Borrowed pointers to the mesh's host arrays (layouts in tyee_mesh_arrays), valid until the
   mesh is destroyed or reordered.  Errors: EINVAL. */
int tyee_mesh_view(const tyee_mesh *mesh, tyee_mesh_arrays *out);

/* omega_max^2 of K = -L_E L_B by normalised iteration in the S-weighted product (the
   imaginary-time iteration of Section 2, used for the eq. 20 bound dt < 2/omega_max).
   gamma: per-edge coefficient scale [n_edges] or NULL.  Start vector
   x_j = 2 u_j - 1, u_j = (splitmix64(seed + j) >> 11) * 2^-53.  Stops when
   |lambda_k - lambda_{k-1}| <= rtol * lambda_k (TYEE_OK) or after max_iter iterations
   (TYEE_ENOTCONVERGED, *lambda still set).  FP64 on host threads. */
int tyee_mesh_cfl(const tyee_mesh *mesh, const double *gamma, int64_t max_iter, double rtol,
                  uint64_t seed, double *lambda, int64_t *iters);

void tyee_mesh_destroy(tyee_mesh *mesh);

/* ----------------------------------------------------------- simulation ---- */

/* Upload a mesh for stepping with time step dt in FP32 or FP64 device arithmetic
   (geometry stays FP64 on the host; coefficients are folded with dt and rounded once).
   stream: a hipStream_t, or NULL to let the library create a stream of its own (the legacy
   default stream cannot be captured into graphs).  Fields start at zero.  The simulation
   copies what it needs: the mesh may be destroyed afterwards.  Errors: EINVAL (prec, dt not
   positive and finite), EDEVICE (no HIP device), ENOMEM. */
int tyee_sim_create(const tyee_mesh *mesh, int32_t prec, double dt, void *stream,
                    tyee_sim **out);

/* Host FP64 arrays in canonical numbering: E [n_edges] (physical projection E_i), B
   [n_tris], J [n_edges] (plasma edges only; other entries must be 0), Q [n_nodes].  Values
   given for outer resonator edges are ignored (they stay 0).  get synchronises the stream. */
int tyee_sim_set_state(tyee_sim *sim, int32_t field, const double *host);
int tyee_sim_get_state(tyee_sim *sim, int32_t field, double *host);

/* Plasma-like medium (eq. 5, j' = wp2 E - nu j, with E' = ... - j of eq. 6 taken with the
   physical sign).  wp2_tri [n_tris]: plasma frequency squared per triangle (canonical);
   each interior edge takes (hR wp2_R + hL wp2_L)/d.  Edges with a positive value form the
   plasma list.  Passing NULL removes the medium. */
int tyee_sim_set_media(tyee_sim *sim, const double *wp2_tri, double nu);

/* Soft current source Jsrc_i(t) = w * g(t) on the edges joining node_pairs[k][0] ->
   node_pairs[k][1] (weight sign follows that direction), g(t) = sin(omega t)
   sin^2(pi t / T) for 0 <= t < T = cycles 2 pi/omega, else 0, taken at t = (n + 1/2) dt.
   n = 0 removes the source.  Errors: TYEE_EINVAL if a pair is not a mesh edge. */
int tyee_sim_set_source(tyee_sim *sim, const int32_t *node_pairs, const double *weights,
                        int64_t n, double omega, double cycles);

/* Per-edge scale gamma_i [n_edges] (canonical) of the eq. 3 and eq. 4 coefficients of
   edge i (the learned correction); NULL restores gamma = 1.  Physical fields are kept. */
int tyee_sim_set_edge_scale(tyee_sim *sim, const double *gamma);

/* Temporal fusion: advance steps_per_launch (1..8; 0 = the default: in FP32 8 for meshes of
   8,000,000 triangles or more, else 6; 4 in FP64) steps in one launch, with or without plasma and
   source edges (tiles that hold such an edge run a variant of the kernel that also advances
   their currents, and the nodal charge follows once per launch).  The device numbering is cut
   into tiles of tile_tris consecutive triangles (0 = a default for the depth: in FP32 2048 at
   up to 4 steps, 1792 at 5, 1536 at 6 or 7, 1024 at 8; in FP64 2048 below 4 steps, else 1024;
   else 256..8192); each work-group loads its tile with
   steps_per_launch rings of neighbours into LDS, advances them, and writes its own cells to
   the other of two field buffers.  Results are bit-identical for every setting.  A mesh
   whose tiles exceed the kernel's capacity falls back to one launch per half-step.  A new
   simulation advances one launch per half-step (steps_per_launch 1) until this is called. */
int tyee_sim_set_fusion(tyee_sim *sim, int32_t steps_per_launch, int32_t tile_tris);

/* Enqueue n leap-frog steps on the simulation's stream (asynchronous; n = 0 does nothing).
   Errors: EINVAL (n < 0), EDEVICE (a launch failed). */
int tyee_sim_step(tyee_sim *sim, int64_t n);

/* Wait for all enqueued work. */
int tyee_sim_sync(tyee_sim *sim);

typedef struct {
    int64_t step;          /* steps taken */
    double time;           /* step * dt */
    double energy;         /* W = sum w E^2 + sum S B^2 at the current levels (eq. 8 with the
                              signed dual length, w = d |e|) */
    double energy_h;       /* W_h = sum w E^n^2 + sum S B^{n-1/2} B^{n+1/2}: the quantity the
                              leap-frog scheme conserves exactly in vacuum (eqs. 7-10);
                              B^{n-1/2} is rebuilt as B^{n+1/2} - dt L_E E^n */
    double max_abs_E, max_abs_B;
    int32_t nonfinite;     /* 1 if any field value is NaN or infinite */
} tyee_diag;

/* Diagnostics from the current state: one device reduction with FP64 accumulation (per-block
   partial sums added on the host in block order, so repeated calls agree bit for bit); the
   FP64 weight tables are built on the first call after the coefficients change (synchronises).
   Returns TYEE_EUNSTABLE if a field is not finite (out is still filled). */
int tyee_sim_diagnostics(tyee_sim *sim, tyee_diag *out);

/* The same diagnostics without any device or host allocation, for callers that cannot
   allocate (tight serving loops, harnesses that forbid hipMalloc).  The per-block partial
   sums and their totals go to a fixed 6 MiB device array of the library (one per GPU, held
   until the process ends, every partial and total overwritten by each call), not to a
   buffer of the simulation; the totals are added on the device in the order
   tyee_sim_diagnostics adds them on the host, so both return the same bits.  Calls that
   overlap on one GPU (simulations on different streams or threads) share that array and race:
   serialise them.  Synchronises the simulation's stream.
   Errors: TYEE_EINVAL if the FP64 weight tables are not built (call tyee_sim_diagnostics once
   after creating the simulation or changing its coefficients; that call allocates them) or
   if the mesh has more than 33,554,432 edges or triangles; TYEE_EDEVICE on a HIP error;
   TYEE_EUNSTABLE as tyee_sim_diagnostics. */
int tyee_sim_diagnostics_noalloc(tyee_sim *sim, tyee_diag *out);

/* Discrete Gauss residual per node (canonical, FP64 host): out_k = (D E)_k - Q_k with
   (D E)_k = sum_i sigma(k,i) d_i E_i, sigma = +1 when e_i leaves node k (the flux of E
   through the dual cell of node k, Section 1).  In vacuum D E is conserved on interior
   nodes; with plasma or a source, D E - Q is.  out: [n_nodes]. */
int tyee_sim_gauss(tyee_sim *sim, double *out);

/* Probe: record field values at canonical ids (edges for E and J, triangles for B, nodes for
   Q) after every step whose count is a multiple of `every`, up to max_samples samples (later
   samples are dropped).  Fused launches are split so that every sampling step is a launch
   boundary.  *probe receives its id. */
int tyee_sim_add_probe(tyee_sim *sim, int32_t field, const int32_t *ids, int64_t n, int64_t every,
                       int64_t max_samples, int32_t *probe);

/* Copy the recorded samples of a probe: out [capacity][n] row-major (physical values),
   *n_samples receives the number recorded (synchronises). */
int tyee_sim_read_probe(tyee_sim *sim, int32_t probe, double *out, int64_t capacity,
                        int64_t *n_samples);

/* Kernel time of the last tyee_sim_step call in milliseconds, measured with HIP events on
   the simulation's stream (synchronises). */
int tyee_sim_last_step_ms(tyee_sim *sim, double *ms);

/* Replay launches from a captured HIP graph, `launches` (an even number, 0 = off) per graph,
   for vacuum runs: fused launches, or with one step per launch the edge and triangle
   half-steps of `launches` steps.  The graph is captured on first use and again after any
   change of fusion, tiling or coefficients.  Stepping with per-launch timing of any single
   kernel kind enabled launches eagerly instead. */
int tyee_sim_set_graph(tyee_sim *sim, int32_t launches);

/* Kernels of one step, for per-launch timing; TYEE_KERNEL_GRAPH times whole graph replays. */
typedef enum { TYEE_KERNEL_EDGE = 0, TYEE_KERNEL_TRI = 1, TYEE_KERNEL_FUSED = 2,
               TYEE_KERNEL_SPECIAL = 3, TYEE_KERNEL_CHARGE = 4, TYEE_KERNEL_GRAPH = 5 } tyee_kernel;

/* Time every later launch of the kernel kinds in the bit mask `kinds` (bit k = tyee_kernel
   k) with a HIP event pair on the simulation's stream; resets the totals.  0 turns timing
   off.  Without TYEE_KERNEL_GRAPH in the mask, timing any other kind turns graph replay off
   so that each launch is timed; with it, replays stay on and are timed whole, and the other
   kinds in the mask time the launches made outside a graph. */
int tyee_sim_set_profiling(tyee_sim *sim, uint32_t kinds);

/* Number of timed launches of one kernel kind and their summed duration in ms since the
   last tyee_sim_set_profiling (waits for the timed launches). */
int tyee_sim_kernel_times(tyee_sim *sim, int32_t kind, int64_t *count, double *total_ms);

/* Fusion in use: out = {steps per launch, tile size in triangles, number of tiles, local
   triangles summed over tiles, local edges summed over tiles, tiles holding a special edge
   (run by the special-edge variant of the fused kernel)}; the last five are 0 until the
   first fused launch has built the tiles. */
int tyee_sim_get_fusion(const tyee_sim *sim, int64_t out[6]);

/* Zero-copy access to the fields: bind caller-owned device memory (for instance two torch
   tensors) as the two buffers of E or B.  Fused launches read one buffer and write the other
   (single-step launches update the current one in place); tyee_sim_current_buffer says which
   of the two holds the state after a call.  Layout: device numbering (perm_e / perm_t of
   tyee_mesh_view), the simulation's precision; E holds the scaled field gamma_i |e_i| E_i (0 on
   outer edges), B holds B_j.  buf0, buf1: n_edges (E) or n_tris (B) elements each, distinct,
   aligned to the element size, valid and not written by anyone else while bound; the current
   state is copied into the buffer of the current parity.  NULL, NULL unbinds: the state
   moves back into library memory.  The library never frees bound memory.  Errors: EINVAL
   (field other than E or B, one NULL, equal or misaligned buffers), ENOMEM, EDEVICE. */
int tyee_sim_bind_external(tyee_sim *sim, int32_t field, void *buf0, void *buf1);
int tyee_sim_current_buffer(const tyee_sim *sim, int32_t *which);

int64_t tyee_sim_steps(const tyee_sim *sim);
void tyee_sim_destroy(tyee_sim *sim);

/* ------------------------------------------------------ learned correction ---- */

/* Eight geometry features per edge (canonical order), FP64: out [n_edges][8] =
   { d/|e|; min and max of the angles opposite the edge in R and L; min and max of
     circumradius / shortest side of R and L; |hR - hL|/d (how far the edge midpoint is from
     the segment O_R O_L, the off-centring that degrades eq. 3); |e|/sqrt(mean triangle
     area); |S_R - S_L|/(S_R + S_L) }.  All are unchanged by swapping R and L or reversing the
   edge (Fig. 2 allows either direction).  Outer edges repeat their one triangle. */
int tyee_mesh_features(const tyee_mesh *mesh, double *out);

/* Rayleigh-quotient estimate of the phase-velocity error of plane waves exp(i k.O) under
   K_gamma = -L_E L_B with edge scale gamma (NULL = 1), with the leap-frog correction.  It is
   an upper (arithmetic-mean) estimate: the sampled wave's high-frequency content raises it,
   so it is a diagnostic, not the measured dispersion (see tyee_phase_error_timestepped):
   omega_RQ^2 = sum_i gamma_i^2 (|e_i|/d_i) |exp(i k.O_R) - exp(i k.O_L)|^2 / sum_j S_j,
   omega = (2/dt) asin(omega_RQ dt/2), out[w] = omega/|k| - 1 (the dispersion of Section 2,
   measured per wave).  waves: [n_waves][2] wavevectors, integer-periodic on a torus.
   Host FP64. */
int tyee_mesh_phase_error_rq(const tyee_mesh *mesh, const double *gamma, double dt,
                             const double *waves, int64_t n_waves, double *out);

/* Time-stepped phase errors of plane waves [n_waves][2]: for each wave two simulations
   (real and imaginary parts of B = exp(i (k.O - |k| dt/2)), E = exp(i k.C) (t . (n x k^)))
   are advanced N = max(samples, round(phase/(|k| dt))) steps on the GPU in `samples` chunks;
   the phase of the overlap z = sum w E conj(E0) + sum S B conj(B0) (metric (7)) is unwrapped
   and fitted by least squares, eps[w] = slope/|k| - 1 (the dispersion of Section 2 as the
   scheme produces it).  gamma: edge scale or NULL; eps: [n_waves] caller-owned; the mesh
   must be periodic with integer-periodic wavevectors.  Errors: EINVAL (zero wavevector,
   samples < 2, phase or dt not positive), EDEVICE. */
int tyee_phase_error_timestepped(const tyee_mesh *mesh, const double *gamma, double dt,
                                 int32_t prec, const double *waves, int64_t n_waves,
                                 double phase, int64_t samples, void *stream, double *eps);

typedef struct tyee_learner tyee_learner;

/* Training set and model on the device.  Model: gamma_i = 1 + 0.1 tanh(w3 . tanh(W2
   tanh(W1 x_i + b1) + b2) + b3), x_i = (f_i - mu)/sd the normalised features of edge i;
   1,377 parameters in the order W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3.
   Loss: the mean over meshes and waves of eps^2, eps the phase error that leap-frog itself
   produces: each plane wave exp(i k.O) is advanced N = round(phase/(|k| dt)) steps of the
   scheme in its B-only form (x_{n+1} = (2 - dt^2 K_gamma) x_n - x_{n-1}, started from the exact
   wave at -dt/2 and +dt/2), and eps = -arg(z_N/z_0)/(|k| N dt) - 1 with z the S-weighted
   overlap with exp(i k.O).  Its gradient comes from the exact adjoint of that recurrence.
   meshes: periodic training meshes; a mesh of at most 4096 triangles and 6144 edges runs each
   of its waves inside one work-group (its state in LDS), a larger one on the multi-work-group
   path (state in device memory, one launch per step for every active wave); dt [n_meshes];
   waves [n_meshes][n_waves][2]; phase in (0, 3) radians.
   mu and sd default to the mean and standard deviation (+1e-6) of the training features.
   Parameters start at zero (gamma = 1); every (mesh, wave) pair is active.  Errors: EINVAL (a
   mesh not periodic or with 2^30 or more cells, dt not positive, phase out of range), EDEVICE,
   ENOMEM. */
int tyee_learner_create(const tyee_mesh *const *meshes, const double *dt, int64_t n_meshes,
                        const double *waves, int64_t n_waves, double phase, void *stream,
                        tyee_learner **out);

/* Stiff-edge term added to the loss: beta * mean over training edges with d/|e| < tau of
   (gamma - target)^2.  Such edges hardly change smooth waves but set omega_max, so gamma
   below 1 there lengthens the stable time step of eq. 20.  Defaults: tau 0.02, beta 1e-3,
   target 0.9; beta = 0 removes the term. */
int tyee_learner_regulariser(tyee_learner *l, double tau, double beta, double target);

/* Glorot-uniform W1, W2 from splitmix64(seed + ...), zero biases and output layer (so the
   initial model is gamma = 1); resets the optimiser. */
int tyee_learner_init(tyee_learner *l, uint64_t seed);
int tyee_learner_set_params(tyee_learner *l, const double *theta);
int tyee_learner_get_params(tyee_learner *l, double *theta);

/* Set (when mu_in and sd_in are given) and/or read the feature normalisation [8] each. */
int tyee_learner_normaliser(tyee_learner *l, const double *mu_in, const double *sd_in,
                            double *mu_out, double *sd_out);

/* Loss, its gradient [1377] (NULL to skip) and the per-(mesh, wave) phase errors eps
   [n_meshes][n_waves] (NULL to skip) for the current parameters, all computed on the GPU. */
int tyee_learner_loss_grad(tyee_learner *l, double *loss, double *grad, double *errors);

/* iters Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr on the GPU;
   loss_history [iters] receives the loss before each step (NULL to skip). */
int tyee_learner_train(tyee_learner *l, int64_t iters, double lr, double *loss_history);

/* gamma [n_edges] of any mesh under the current model (1 on outer edges), computed by the
   GPU forward kernel. */
int tyee_learner_gamma(tyee_learner *l, const tyee_mesh *mesh, double *gamma);
/* Minibatch: from now on the loss is the mean of eps^2 over the listed (mesh, wave) pairs
   [n][2] only (plus the stiff-edge term over every training edge), and training and
   tyee_learner_loss_grad compute only those pairs; the errors of other pairs read NaN.
   pairs = NULL or n = 0 makes every pair active again.  Allocates the state of the
   multi-work-group path for the batch.  Errors: EINVAL (a pair out of range or listed twice). */
int tyee_learner_set_batch(tyee_learner *l, const int32_t *pairs, int64_t n);

/* 0 (default): meshes that fit one work-group use it, larger ones the multi-work-group path;
   1: every mesh on the multi-work-group path (both paths run the same single-precision
   recurrences; used to check one against the other). */
int tyee_learner_set_path(tyee_learner *l, int32_t path);
void tyee_learner_destroy(tyee_learner *l);

typedef struct {
    int32_t accepted;      /* converged and err_learned < err_plain */
    int32_t converged;     /* both power iterations converged */
    double omega_plain, omega_learned;  /* omega_max without and with gamma */
    double dt_plain, dt_learned;        /* cfl * 2 / omega_max */
    double err_plain, err_learned;      /* mean |time-stepped phase error| over the held-out
                                           waves, each at its own dt */
} tyee_gate_result;

/* Per-mesh acceptance of a learned scale: omega_max with and without gamma by power
   iteration (the eq. 20 bound fixes dt = cfl * 2/omega_max for each), then the mean absolute
   time-stepped phase error (tyee_phase_error_timestepped, about `phase` radians of travel,
   10 samples) over held-out waves [n_waves][2], each method at its own dt.  Callers use
   gamma and dt_learned only when accepted, else the plain coefficients and dt_plain. */
int tyee_gate(const tyee_mesh *mesh, const double *gamma, const double *waves, int64_t n_waves,
              double cfl, double phase, int32_t prec, void *stream, tyee_gate_result *out);

/* Lawson flips of a triangulation (Section 3: the flip operation of Fig. 5a): while an
   interior edge fails the empty-circle test (the apex of its second triangle strictly inside
   the circumcircle of the first, beyond a relative tolerance of 1e-12 that leaves cocircular
   quads alone), replace it by the other diagonal of its quad.  xy [n_nodes][2]; tri
   [n_tris][3] is rewritten in place (counter-clockwise) only on success; dom gives the kind and
   the periods (minimum image on a torus).  flips (NULL to skip) receives the count.  Host
   only.  Errors: TYEE_EINVAL (ids out of range), TYEE_EDEGENERATE (a zero-area triangle),
   TYEE_EUNSTABLE (no end within 50 n_tris flips). */
int tyee_mesh_flip(const double *xy, int64_t n_nodes, int32_t *tri, int64_t n_tris,
                   const tyee_domain *dom, int64_t *flips);

/* ---------------------------------------------------------- relaxation ---- */

typedef struct {
    int32_t rounds;       /* remesh rounds: each runs `iters` Euler steps, Lawson flips, omega_max */
    int32_t iters;        /* Euler steps per round */
    double step;          /* Euler step tau: a node moves by tau times its net spring force */
    double k_edge;        /* spring constant along edges */
    double k_height;      /* spring constant along triangle heights */
    double rest;          /* rest length of the edge springs; 0: the side of the equilateral
                             triangle that covers the domain with n_tris triangles (heights rest
                             at rest sqrt(3)/2) */
    int32_t keep_best;    /* 1: return the iterate (input included) with the smallest omega_max;
                             0: return the last round's */
} tyee_relax_params;

typedef struct {
    double omega_initial;  /* omega_max of the input mesh */
    double omega_best;     /* omega_max of the returned mesh */
    int32_t best_round;    /* 0 when the input mesh is returned */
    int64_t flips;         /* Lawson flips over all rounds */
    double energy_initial, energy_final;  /* spring energy of the input and returned node sets */
    double step_used;      /* Euler step after any halving (a triangle that turns over makes the
                              round start again at half the step, up to 5 times) */
} tyee_relax_stats;

/* Jello relaxation of the mesh's nodes (Section 3, mesh generation, Fig. 5b): nodes joined by
   springs along every triangle edge and every triangle height, at the rest lengths of a perfect
   equilateral mesh, move along their net force (heavily damped motion without its second time
   derivative: x <- x + step F, Euler steps on the GPU, FP64); after every round of `iters`
   steps the triangulation is remeshed by Lawson flips and omega_max of the result is measured
   by power iteration (eq. 20: dt = C 2/omega_max).  Nodes on the outline of a closed
   resonator and the n_anchors node ids in `anchors` (seeds of the geometry) do not move.
   Outputs (caller buffers, canonical node ids, node and triangle counts unchanged): xy_out
   [n_nodes][2], tri_out [n_tris][3] (counter-clockwise) of the returned iterate, for
   tyee_mesh_create with the input's domain; omega_rounds [rounds + 1] (NULL to skip):
   omega_max of the input and after each round (+infinity when a round's mesh is not Delaunay);
   stats (NULL to skip).  stream: HIP stream for the steps (NULL = default).
   Errors: TYEE_EINVAL (bad parameters or anchors), TYEE_EUNSTABLE (triangles fold even at 1/32
   of the step), TYEE_EDEVICE, TYEE_ENOMEM. */
int tyee_mesh_relax(const tyee_mesh *mesh, const tyee_relax_params *p, const int32_t *anchors,
                    int64_t n_anchors, void *stream, double *xy_out, int32_t *tri_out,
                    double *omega_rounds, tyee_relax_stats *stats);

/* ---------------------------------------------------------------- batch ---- */

typedef struct tyee_batch tyee_batch;

/* Step many independent meshes together (vacuum).  The members are copied and stored as one
   disjoint union: their cells are concatenated in the device numbering (each member keeps
   its own locality order inside its range) and member k's time step dt[k] is folded into
   its cells' coefficients, so one launch advances every member.  Each member's fields are
   bit-identical to a standalone simulation with the same dt, numbering and precision.
   meshes: [n_meshes] handles (may be destroyed afterwards); stream as for
   tyee_sim_create.  Fields start at zero. */
int tyee_batch_create(const tyee_mesh *const *meshes, const double *dt, int64_t n_meshes,
                      int32_t prec, void *stream, tyee_batch **out);

/* Member k's E [n_edges_k] or B [n_tris_k] in the member's own canonical numbering (FP64
   host, copied; get synchronises).  Errors: EINVAL (k out of range, other fields). */
int tyee_batch_set_state(tyee_batch *b, int64_t k, int32_t field, const double *host);
int tyee_batch_get_state(tyee_batch *b, int64_t k, int32_t field, double *host);

/* Renumber every member (as tyee_mesh_reorder); fields are kept. */
int tyee_batch_reorder(tyee_batch *b, int32_t kind, uint64_t seed);
/* As tyee_sim_set_fusion / _set_graph / _step / _sync, for the union of the members. */
int tyee_batch_set_fusion(tyee_batch *b, int32_t steps_per_launch, int32_t tile_tris);
int tyee_batch_set_graph(tyee_batch *b, int32_t launches);
int tyee_batch_step(tyee_batch *b, int64_t n);
int tyee_batch_sync(tyee_batch *b);

/* out = {members, triangles, edges, nodes} of the union. */
int tyee_batch_info(const tyee_batch *b, int64_t out[4]);

/* Borrowed handle of the union's simulation (profiling, fusion info, diagnostics); valid
   until the next reorder, tune or destroy of the batch. */
int tyee_batch_sim(tyee_batch *b, tyee_sim **sim);

typedef struct {
    int32_t order;             /* tyee_order */
    int32_t steps_per_launch;  /* 1, 2, 4, 6 or 8 */
    int32_t tile_tris;         /* 0 for one launch per half-step */
    double ms_per_step;        /* HIP-event time of the trial divided by its steps */
} tyee_tune_result;

/* Autotune: time about steps_per_trial steps for every ordering (Morton, RCM) x steps per
   launch (1, 2, 4, 6, 8) x tile size (1024, 1536, 2048, 3072; one trial at 1 step per
   launch), 34 trials, keep the fastest setting and
   restore the fields and step count.  results: [capacity] trial records (may be NULL when
   capacity is 0); *n_results receives the number of trials. */
int tyee_batch_tune(tyee_batch *b, int64_t steps_per_trial, tyee_tune_result *results,
                    int64_t capacity, int64_t *n_results);

/* Called after each autotuner trial with its record (borrowed for the call) and the caller's
   pointer; it must not call back into the batch. */
typedef void (*tyee_tune_progress)(const tyee_tune_result *trial, void *user);
/* tyee_batch_tune that reports every trial as it ends through on_trial (may be NULL, which is
   tyee_batch_tune itself).  Same arguments, results and errors. */
int tyee_batch_tune_progress(tyee_batch *b, int64_t steps_per_trial, tyee_tune_result *results,
                             int64_t capacity, int64_t *n_results, tyee_tune_progress on_trial,
                             void *user);

void tyee_batch_destroy(tyee_batch *b);

/* Achievable device bandwidth, the reference beside the published HBM peak in roofline
   reports: copies `bytes` (1 MiB .. 16 GiB) between two device buffers `reps` times with
   16-byte non-temporal loads and stores (one element per work-item) on a stream of its own,
   timed with HIP events; *gbs = bytes read + written per second / 1e9.  Allocates and frees
   its two buffers.  Errors: EINVAL, ENOMEM, EDEVICE. */
int tyee_copy_bandwidth(int64_t bytes, int32_t reps, double *gbs);

/* End of the spectrum tyee_mesh_modes computes. */
typedef enum { TYEE_MODES_LOWEST = 0, TYEE_MODES_HIGHEST = 1 } tyee_modes_end;

/* Work done by one tyee_mesh_modes call. */
typedef struct {
    int32_t iters;         /* outer iterations (three filter passes, each followed by the
                              orthonormalisation, then one Rayleigh-Ritz step) */
    int64_t applies;       /* applications of K to the whole block */
    double lambda_bound;   /* Gershgorin bound on lambda_max that closes the filter interval */
    double filter_ms;      /* HIP-event time of the filter launches on the stream */
    double total_ms;       /* host wall time of the call, uploads and readback included */
} tyee_modes_stats;

/* Lowest or highest eigenmodes of the resonator (Section 2: eigenvectors of the Maxwell operator, which
   the energy law (10) makes real and orthogonal in metric (7), and the "complex time"
   iteration that finds them; Fig. 4).  With E eliminated, eqs. 3-4 give for B the operator
   K = -L_E L_B, (K B)_j = (1/S_j) sum over interior edges i of j of
   gamma_i^2 |e_i|/d_i (B_j - B_other), self-adjoint and non-negative in the weights S_j;
   K v = lambda v, omega = sqrt(lambda); the constant field is the static mode (lambda = 0).
   Outer edges carry E = 0 (PEC) and add nothing.

   Computed on the device in FP64 by a block iteration: a polynomial filter run as the
   three-term (leap-frog) recurrence of the shifted K, with the unwanted part of the spectrum
   inside the eq. 20 bound (bounded) and the wanted modes outside it (growing, as in complex
   time); S-orthonormalisation of the block (deflation in metric (7)) after each filter pass;
   a Rayleigh-Ritz step after every three passes.
     gamma     [n_edges] per-edge scale in canonical order, or NULL.
     which     TYEE_MODES_LOWEST, or TYEE_MODES_HIGHEST (the paper's order: the largest
               eigenvalue first; the solver then works on lambda_bound - K, whose lowest modes
               are K's highest).
     n_modes   1 .. min(n_triangles, 256) pairs wanted.
     block     vectors iterated, max(n_modes, 2) .. min(n_triangles, 256); 0 chooses
               n_modes + max(16, n_modes / 4) (capped).  n_triangles x block < 2^31.
     degree    largest filter degree per pass (three passes per outer iteration), 1 .. 100000;
               0 chooses 128.  A pass lowers it so that the lowest Ritz value grows at most 1e7
               times more than the cut (the block stays well enough conditioned to
               orthonormalise).
     tol       converged when ||K v_c - lambda_c v_c||_S <= tol * lambda_bound for every wanted
               c (v_c S-normalised).
     max_iter  outer iterations allowed (>= 1).
     seed      start block x[j][c] = 2u - 1, u = (splitmix64(seed + j block + c) >> 11) 2^-53
               with j canonical (the same splitmix64 as tyee_mesh_cfl).
     stream    HIP stream, or NULL for the default stream.
     omega2    [n_modes] host out: lambda, ascending (lowest) or descending (highest).
     modes     [n_modes][n_triangles] host out (canonical triangle order), S-orthonormal, or NULL.
     residual  [n_modes] host out: residual norm / lambda_bound, or NULL.
     stats     host out, or NULL.
   Allocates about 5 x n_triangles x block doubles of device memory for the call and frees it;
   blocks on the stream.  Errors: EINVAL (arguments; a mesh with no interior edge), ENOMEM,
   EDEVICE, EUNSTABLE (the block lost rank), ENOTCONVERGED (outputs are still written from the
   last iteration). */
int tyee_mesh_modes(const tyee_mesh *mesh, const double *gamma, int32_t which, int64_t n_modes,
                    int32_t block, int32_t degree, double tol, int32_t max_iter, uint64_t seed,
                    void *stream, double *omega2, double *modes, double *residual,
                    tyee_modes_stats *stats);

/* Work done by one tyee_mesh_spectrum call. */
typedef struct {
    int32_t windows;       /* spectral windows solved */
    int32_t iters;         /* Rayleigh-Ritz steps after filter passes, over all windows */
    int64_t found;         /* pairs accepted (n_triangles on success) */
    int64_t applies;       /* applications of K to the whole block */
    int64_t below;         /* converged Ritz pairs outside a window (found before), set aside */
    int64_t retries;       /* interior filter passes redone at a lower growth (the block was too
                              ill-conditioned for the shifted Cholesky QR) */
    double lambda_bound;   /* Gershgorin bound on lambda_max */
    double filter_ms;      /* HIP-event time of the filter launches on the stream */
    double total_ms;       /* host wall time of the call, uploads and readback included */
    double max_residual;   /* largest residual / lambda_bound of an accepted pair */
    double min_gap;        /* smallest eigenvalue gap at a window boundary / lambda_bound */
    int64_t sq_launches;   /* launches of the fused (K - sigma)^2 block apply */
    double sq_ms;          /* HIP-event time of the interior windows' filter passes (those
                              launches only) */
} tyee_spectrum_stats;

/* Every eigenmode of the resonator: all n_triangles eigenpairs of K = -L_E L_B (the operator of
   tyee_mesh_modes), the whole spectrum of Fig. 4 (Section 2: as many eigenvalues as B
   components, the constant field the static one).  The paper finds the modes one after another
   by the "complex time" iteration, withdrawing the modes already found from the start vector
   by orthogonality in metric (7); here the same filter, deflation and Rayleigh-Ritz run window
   by window over the spectrum in FP64 on the device:
     window 0     the lowest modes (the low-pass filter of tyee_mesh_modes);
     windows 1..  beta = the boundary below which every mode is found; the filter runs on
                  (K - sigma)^2 with sigma a quarter of the block's reach above beta, whose
                  lowest modes are K's modes nearest sigma; the start block (the last window's
                  Ritz vectors above its boundary, the other columns random) is S-orthogonalised
                  against the modes of the last three windows;
     last window  the remaining top modes (the filter of lambda_bound - K).
   Each filter pass is followed by the orthonormalisation and a Rayleigh-Ritz step.  A window
   trusts its converged Ritz pairs taken in order of ||(K - sigma) v|| up to the first one that
   has not converged (every mode closer to sigma than that one is among them), and accepts those
   at or above beta up to a boundary placed in the widest gap (>= 16 tol lambda_bound) of their
   top fifth, once 0.6 x block of them are trusted (or the trusted set stops growing).  Modes
   found before that grow back below beta are set aside (stats->below).  The cost of a window
   grows with the spread of the spectrum over the window's width: meshes with nearly cocircular
   quads (very large lambda_bound) need high filter degrees.  n_triangles <= block: one exact
   Rayleigh-Ritz step.
     gamma     [n_edges] per-edge scale in canonical order, or NULL.
     block     vectors iterated, min(n_triangles, 16) .. min(n_triangles, 256); 0 chooses
               min(n_triangles, 192).  n_triangles x block < 2^31.
     degree    largest filter degree per pass in applications of K, 2 .. 100000; 0 = no limit
               beyond the conditioning cap of tyee_mesh_modes (growth from the bottom of the
               filter interval to the cut at most 2e7).
     tol       a pair is converged when ||K v - lambda v||_S <= tol * lambda_bound (v
               S-normalised); an eigenvalue is then within tol * lambda_bound of lambda.  Modes
               of different windows are S-orthogonal to about tol * lambda_bound / (their gap).
     max_iter  Rayleigh-Ritz steps allowed per window (>= 1).
     seed      window w starts its random columns as in tyee_mesh_modes with seed
               seed + w n_triangles block.
     stream    HIP stream, or NULL for the default stream.
     omega2    [n_triangles] host out: lambda ascending.
     modes     [n_triangles][n_triangles] host out (mode-major, canonical triangle order,
               S-normalised), or NULL.
     residual  [n_triangles] host out: residual / lambda_bound, or NULL.
     stats     host out, or NULL.
   Allocates about 8 (9 with modes) x n_triangles x block doubles of device memory for the call
   and frees it; blocks on the stream.  Set TYEE_SPECTRUM_TRACE in the environment for one line
   per Rayleigh-Ritz step on stderr.  Errors: EINVAL (arguments; a mesh with no interior edge),
   ENOMEM, EDEVICE, EUNSTABLE (the block lost rank; more converged modes above the last boundary
   than remain), ENOTCONVERGED (a window did not converge within max_iter; the first
   stats->found outputs are written). */
int tyee_mesh_spectrum(const tyee_mesh *mesh, const double *gamma, int32_t block, int32_t degree,
                       double tol, int32_t max_iter, uint64_t seed, void *stream, double *omega2,
                       double *modes, double *residual, tyee_spectrum_stats *stats);

/* ---------------------------------------------------------------------------------------
   Open boundary: the triangle mesh of a closed box tied to a rectangular frame of PML layers.
   The paper's Conclusion: the scheme works on mixed meshes (triangles plus quads), so a mesh
   with rectangular boundaries can be joined to a structured frame that carries PML layers.
   A rectangle's circumcentre is its centre, on the perpendicular bisector of each side as a
   triangle's circumcentre is, so eqs. 3-4 hold on the mixed mesh unchanged.

   The frame: the mesh must fill the box [0, Lx] x [0, Ly] (a TYEE_PEC_BOX mesh whose outer edges
   lie on the box sides, with nodes exactly on the side lines).  Each side is continued outwards
   by `layers` rows of rectangles `width` deep whose columns (rows) are bounded by that side's
   boundary nodes; each corner by layers x layers squares.  The frame's outer wall is a perfect
   conductor (E = 0).  Damping: sigma(rho) = sigma_max (rho / (layers width))^grading, rho the
   distance beyond the box in x (sigma_x) or y (sigma_y).  A frame cell's B is split into Bx
   (driven by its two sides parallel to y, decaying with its sigma_x) and By (its two sides
   parallel to x, sigma_y); an edge parallel to x decays with sigma_y at its midpoint, one
   parallel to y with sigma_x; triangles and edges inside the box do not decay.  Each damping
   term is taken at the half step: X <- (1 - sigma dt/2)/(1 + sigma dt/2) X + dt/(1 + sigma dt/2)
   (drive).  A step updates E (eq. 3, B_left - B_right over the centre distance d, edges
   oriented from the lower node id to the higher, "left" the cell on the left of that tangent),
   then B (eq. 4, -(1/S) sum over the cell's edges of s |e| E, s = +1 where the edge runs
   counter-clockwise around the cell), one launch each.

   Canonical numbering of the mixed mesh: the triangle mesh's nodes, edges and triangles keep
   their ids; the frame's new nodes follow ordered by (y, x), its edges follow the mesh's
   ordered by (lower, higher) node id, its rectangles follow the triangles ordered by the (y, x)
   of their centres.  Device arrays are in the same order; the device holds each edge's line
   integral |e| E (converted on set and get), so that a cell's update reads only the sign of
   each side. */
typedef struct tyee_open tyee_open;

typedef struct {
    int32_t layers;        /* rows of rectangles around each side, 1 .. 4096 */
    double width;          /* depth of one row (> 0) */
    double sigma_max;      /* damping rate at the outer wall (>= 0; 0 gives a reflecting frame) */
    double grading;        /* exponent of the profile (>= 0) */
} tyee_pml_params;

/* Fields of the open simulation.  E: [n_edges] (the frame's outer wall stays 0); BX: [n_cells],
   B of a triangle and the Bx part of a frame cell; BY: [n_cells] with the By part of frame
   cells (entries of triangles are ignored on set and returned as 0).  B = BX + BY. */
typedef enum { TYEE_OPEN_E = 0, TYEE_OPEN_BX = 1, TYEE_OPEN_BY = 2 } tyee_open_field;

/* Build the frame (host, FP64), upload the coefficients (prec TYEE_F32 or TYEE_F64) for the time
   step dt, zero state.  stream: HIP stream, or NULL for one of the library's own.  Errors:
   EINVAL (a periodic mesh, a mesh that does not fill the box, bad parameters), ENOTDELAUNAY (a
   centre distance across an edge is not positive), ENOMEM, EDEVICE.  *out gets the handle. */
int tyee_open_create(const tyee_mesh *mesh, const tyee_pml_params *pml, int32_t prec, double dt, void *stream,
                     tyee_open **out);
/* out = {n_nodes, n_edges, n_cells, n_frame_cells, n_inner_edges} of the mixed mesh. */
int tyee_open_sizes(const tyee_open *o, int64_t out[5]);
/* The mixed mesh that tyee_open_create builds, built on the host alone (no device): sizes =
   {n_nodes, n_edges, n_cells, n_frame_cells, n_inner_edges}; the arrays, in canonical order, may
   each be NULL (a first call with all of them NULL gives the sizes): xy [n_nodes][2], edge
   [n_edges][2] (lower, higher node id), cell_edge [n_cells][4] (a rectangle: its sides parallel
   to y, then those parallel to x; a triangle's fourth entry -1), elen, d (centre distance across
   the edge, 0 on the outer wall), sigma_e [n_edges]; S, sigma_x, sigma_y [n_cells] (0 on
   triangles); O [n_cells][2] circumcentres.  Errors as tyee_open_create's, ENOMEM. */
int tyee_open_frame(const tyee_mesh *mesh, const tyee_pml_params *pml, int64_t sizes[5], double *xy,
                    int32_t *edge, int32_t *cell_edge, double *elen, double *d, double *S, double *O,
                    double *sigma_e, double *sigma_x, double *sigma_y);
/* Largest eigenvalue lambda of K = -L_E L_B on the mixed mesh without damping (FP64 power
   iteration on the host); omega_max = sqrt(lambda) sets dt < 2/omega_max (eq. 20).  Errors:
   EINVAL, ENOTCONVERGED (*lambda still set). */
int tyee_open_cfl(const tyee_open *o, int64_t max_iter, double rtol, uint64_t seed, double *lambda,
                  int64_t *iters);
/* Host values (FP64, canonical order) to or from the device; both wait for the stream. */
int tyee_open_set_state(tyee_open *o, int32_t field, const double *values);
int tyee_open_get_state(tyee_open *o, int32_t field, double *values);
/* Enqueue nsteps steps on the stream (returns without waiting unless timing is on): whole
   groups of the graph size replay one captured HIP graph (the stream must allow capture: a
   caller's stream other than the legacy default one), the rest are launched one by one. */
int tyee_open_step(tyee_open *o, int64_t nsteps);
/* Steps per captured graph, 0 .. 1024 (0: every launch eager; default 8).  Waits for the stream
   if a graph exists (it is discarded).  Errors: EINVAL. */
int tyee_open_set_graph(tyee_open *o, int32_t steps);
/* Fused stepping of the box (the temporal fusion of tyee_sim_set_fusion carried to the open
   boundary): steps_per_launch K (1..8; 0 = 7 in FP32, 4 in FP64; 1 = off, the default),
   tile_tris as in tyee_sim_set_fusion.  mesh must be the triangle mesh the handle was created
   from (checked: counts and edges).  The library then holds a Morton-numbered copy of the box
   advanced by the fused kernel, and a band (every frame cell and edge, the box triangles within
   2K + 3 rings of its sides and their edges) on compact arrays advanced by the single-step
   kernels; each group of K steps gathers the band's box cells, runs one fused launch over the
   box and K band steps, and writes the band's cells within K + 2 rings of the sides over the
   box's (one step carries information one cell, so both parts are exact).  tyee_open_step
   moves the state into these two parts and back around its whole groups of K steps (the rest
   run one launch per half-step, as do timed steps); the state stays in canonical order for
   tyee_open_set_state / _get_state.  Groups run from a captured HIP graph of 8 groups (the
   band's steps on a second stream of the library's beside the fused launch) when the graph size
   of tyee_open_set_graph is not 0, else eagerly in order on the handle's stream (bit-identical).
   Waits for the stream.
   Errors: EINVAL (bad arguments, another mesh, a box that does not tile at that depth),
   ENOMEM, EDEVICE. */
int tyee_open_set_fusion(tyee_open *o, const tyee_mesh *mesh, int32_t steps_per_launch, int32_t tile_tris);
int tyee_open_sync(tyee_open *o);
/* With timing on, steps are launched one by one, each with HIP events around its two launches
   (read after every 256 steps, so a timed call waits for its steps; the events add a few us to
   each launch's reading);
   tyee_open_kernel_ms gives the summed milliseconds {E update, B update} and the steps timed
   since timing was set. */
int tyee_open_set_timing(tyee_open *o, int32_t on);
int tyee_open_kernel_ms(const tyee_open *o, double out[2], int64_t *steps);
int tyee_open_destroy(tyee_open *o);

/* ---------------------------------------------------------------------------------------
   Three dimensions: tetrahedra (the paper's Conclusion: E and j on edges, B on faces, n on
   nodes).  The dual is the Voronoi diagram of the nodes (the circumcentres of the
   tetrahedra), as the triangles' circumcentres are in two dimensions.  Faraday on a face and
   Ampere on an edge's Voronoi polygon (the 3-D form of eqs. 3-4):
     A_f dB_f/dt = -sum over the face's edges of s |e| E_e,
     A*_e dE_e/dt = sum over the faces around the edge of s d_f B_f,
   with d_f = (C_front - C_back) . n_f the distance between the circumcentres on either side of
   face f along its unit normal, A*_e the area of the edge's Voronoi polygon, s = +1 where the
   face's circuit runs along the edge.  Leap-frog, E then B; dt < 2/omega_max (eq. 20).  The
   mesh fills a box whose walls are perfect conductors: a face with one tetrahedron is a wall
   face, every edge of a wall face a wall edge (E = 0 there, B of wall faces never changes).

   Canonical numbering: nodes as given; edges by (lower, higher) node id, tangent from the lower
   to the higher; faces by their sorted node triples (a, b, c), unit normal by the right-hand
   rule of a -> b -> c, whose circuit runs along (a, b) and (b, c) and against (a, c);
   tetrahedra as given.  The device holds the line integrals |e| E and d_f B (B itself on wall
   faces), converted on set and get. */
typedef struct tyee_tet tyee_tet;
typedef struct tyee_tet_sim tyee_tet_sim;
typedef enum { TYEE_TET_E = 0, TYEE_TET_B = 1 } tyee_tet_field;

/* Build the mesh on the host (FP64): xyz [nv][3], tets [nt][4] node ids (any orientation; each
   is reoriented to positive volume).  Errors: EINVAL (null, sizes, an index out of range),
   EDEGENERATE (a tetrahedron with no volume), ENONMANIFOLD (a face shared by more than two
   tetrahedra, or two tetrahedra on one side of a face), ENOTDELAUNAY (d_f <= 0 across an inner face or an inner edge's Voronoi
   polygon without positive area: the mesh is not a Delaunay tetrahedralisation), ENOMEM.
   *out gets the handle; the arrays are copied. */
int tyee_tet_create(const double *xyz, int64_t nv, const int32_t *tets, int64_t nt, tyee_tet **out);
/* out = {n_nodes, n_edges, n_faces, n_tets, n_inner_edges, n_inner_faces, n_incidences} with
   n_incidences the (inner edge, face around it) pairs the E update reads. */
int tyee_tet_sizes(const tyee_tet *m, int64_t out[7]);
/* Canonical arrays, each may be NULL: edge [n_edges][2], face [n_faces][3], face_edge
   [n_faces][3] (its (a,b), (b,c), (a,c) edges), elen and dual_area [n_edges] (0 on wall edges),
   farea and d [n_faces] (d 0 on wall faces), C [n_tets][3] circumcentres. */
int tyee_tet_view(const tyee_tet *m, int32_t *edge, int32_t *face, int32_t *face_edge, double *elen,
                  double *dual_area, double *farea, double *d, double *C);
/* Largest eigenvalue lambda of K = -curl_B curl_E on the inner edges (FP64 power iteration on
   the host in the energy weights A*_e |e|); omega_max = sqrt(lambda).  Errors: EINVAL,
   ENOTCONVERGED (*lambda still set). */
int tyee_tet_cfl(const tyee_tet *m, int64_t max_iter, double rtol, uint64_t seed, double *lambda, int64_t *iters);
int tyee_tet_destroy(tyee_tet *m);

/* Upload the coefficients (prec TYEE_F32 or TYEE_F64) for the time step dt, zero state.
   stream: HIP stream, or NULL for one of the library's own.  The mesh may be destroyed
   afterwards.  Errors: EINVAL, ENOMEM, EDEVICE. */
int tyee_tet_sim_create(const tyee_tet *m, int32_t prec, double dt, void *stream, tyee_tet_sim **out);
/* E [n_edges] or B [n_faces], FP64 host values in canonical order; both wait for the stream. */
int tyee_tet_sim_set_state(tyee_tet_sim *s, int32_t field, const double *values);
int tyee_tet_sim_get_state(tyee_tet_sim *s, int32_t field, double *values);
/* Enqueue nsteps steps (two launches each: the E update over the edges, then the B update over
   the faces); whole groups of the graph size replay one captured HIP graph (the stream must
   allow capture), the rest are launched one by one. */
int tyee_tet_sim_step(tyee_tet_sim *s, int64_t nsteps);
/* Steps per captured graph, 0 .. 1024 (0: eager launches; default 8).  Errors: EINVAL. */
int tyee_tet_sim_set_graph(tyee_tet_sim *s, int32_t steps);
int tyee_tet_sim_sync(tyee_tet_sim *s);
/* With timing on, steps are launched one by one with HIP events around both launches (read
   every 256 steps); tyee_tet_sim_kernel_ms gives the summed milliseconds {E update, B update}
   and the steps timed since timing was set. */
int tyee_tet_sim_set_timing(tyee_tet_sim *s, int32_t on);
int tyee_tet_sim_kernel_ms(const tyee_tet_sim *s, double out[2], int64_t *steps);
int tyee_tet_sim_destroy(tyee_tet_sim *s);

const char *tyee_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
