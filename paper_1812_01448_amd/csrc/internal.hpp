// Internal declarations shared by the host mesh code and the HIP runtime of libtyee.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "tyee.h"

namespace tyee {

// Host-side mesh: canonical connectivity, FP64 geometry and the device numbering.
struct Mesh {
    int64_t nv = 0, ne = 0, nt = 0, nb = 0;
    bool periodic = false;
    double Lx = 1.0, Ly = 1.0;
    std::vector<double> xy;        // [nv][2]
    std::vector<int32_t> tri;      // [nt][3], counter-clockwise
    std::vector<int32_t> edge;     // [ne][2] (lo, hi)
    std::vector<int32_t> R, L;     // [ne], -1 when absent
    std::vector<int32_t> A;        // [nt][3]
    std::vector<int8_t> sgn;       // [nt][3]
    std::vector<double> evec;      // [ne][2]
    std::vector<double> elen, hR, hL, d;  // [ne]
    std::vector<double> S;         // [nt]
    std::vector<double> O;         // [nt][2]
    std::vector<double> C;         // [ne][2]
    std::vector<uint8_t> node_outer;  // [nv] node touches an outer edge
    std::vector<int32_t> perm_t, perm_e;  // device slot -> canonical id
    int32_t order_kind = TYEE_ORDER_NONE;

    bool interior(int64_t i) const { return R[i] >= 0 && L[i] >= 0; }
};

// Record a message for tyee_last_error() and return code.
int fail(int code, const std::string &msg);
void clear_error();

int build_mesh(const double *xy, int64_t nv, const int32_t *tri, int64_t nt,
               const tyee_domain &dom, Mesh &m);
int reorder_mesh(Mesh &m, int32_t kind, uint64_t seed);
int power_iteration(const Mesh &m, const double *gamma, int64_t max_iter, double rtol,
                    uint64_t seed, double *lambda, int64_t *iters);
uint64_t splitmix64(uint64_t x);
// Lawson flips (Section 3, Fig. 5a) until every interior edge of the counter-clockwise
// triangles passes the empty-circle test; n_flips receives the count.  TYEE_EUNSTABLE when
// max_flips is reached first.
int lawson_flip(const std::vector<double> &xy, std::vector<int32_t> &tri, bool periodic, double Lx, double Ly,
                int64_t nv, int64_t max_flips, int64_t *n_flips);
// Disjoint union of meshes: node, edge and triangle ids of part p are offset by the totals
// of parts 0..p-1, and so are their device numberings (each part keeps its own order).
int merge_meshes(const std::vector<const Mesh *> &parts, Mesh &out);
// Eight geometry features per edge for the learned coefficient scale (see tyee_mesh_features).
constexpr int kFeatures = 8;
void edge_features(const Mesh &m, std::vector<double> &out);
// Minimum-image O_R - O_L per edge (0 on outer edges).
void dual_vectors(const Mesh &m, std::vector<double> &out);
// Plane-wave phase errors from the Rayleigh quotient of K_gamma (host FP64).
void rq_phase_errors(const Mesh &m, const double *gamma, double dt, const double *waves, int64_t n_waves,
                     double *out);
uint32_t morton_key(uint32_t qx, uint32_t qz);

// Run fn(begin, end) over [0, n) on the host's hardware threads in 256 fixed contiguous
// chunks (results never depend on the thread count when fn writes disjoint outputs).
// `work` (default n) is the total cost in element units; small jobs run on the caller.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t work = -1);

}  // namespace tyee

struct tyee_mesh {
    tyee::Mesh m;
};
