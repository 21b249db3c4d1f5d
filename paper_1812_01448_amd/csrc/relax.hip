// Jello relaxation of a mesh's nodes (Section 3 of arXiv:1812.01448, Fig. 5b).
//
// The node cloud is treated as nodes joined by springs along every triangle edge and along
// every triangle height, at the rest lengths of a perfect mesh of equilateral triangles that
// covers the domain with the same number of triangles.  The motion is heavily damped and its
// second time derivative dropped, so every free node moves along its net spring force; Euler
// steps integrate that.  Between rounds of steps the triangulation is remeshed by Lawson
// flips (a flip replaces the diagonal of two triangles whose quad fails the empty-circle
// test), nodes of the closed resonator's outline and any caller-given seeds stay anchored, and
// the stable time step of the remeshed mesh is measured: omega_max by power iteration
// (eq. 20).  The iterate with the smallest omega_max is returned.
//
// Energy: E = sum over edges of k_e/2 (l - a)^2 + sum over triangles and their three vertices
// of k_h/2 (h - a sqrt(3)/2)^2, h the distance of the vertex from the opposite side.  The GPU
// step is one work-item per node gathering the forces -dE/dx of its incident edges and
// triangles (node -> edge and node -> triangle lists, so the sum has a fixed order and no
// atomics), then the Euler update; positions are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "internal.hpp"
#include "sim.hpp"

namespace tyee {
namespace {

constexpr int kRelaxThreads = 256;

struct RelaxGeom {
    int periodic;
    double Lx, Ly;
    double a0, h0, k_e, k_h, tau;
};

__device__ __forceinline__ double mi(double d, double L, int periodic) {
    return periodic ? d - L * rint(d / L) : d;
}

__device__ __forceinline__ double wrap(double x, double L) { return x - L * floor(x / L); }

// One Euler step of every node: x <- x + tau F(x) (anchored nodes keep their place).
// e_off/e_other: node -> other ends of its edges; t_off/t_ref: node -> (triangle << 2 | local
// vertex) of its triangles; tri: counter-clockwise vertices.
__global__ __launch_bounds__(kRelaxThreads) void k_relax_step(int nv, RelaxGeom G, const double2 *__restrict__ xin,
                                                              double2 *__restrict__ xout,
                                                              const int32_t *__restrict__ e_off,
                                                              const int32_t *__restrict__ e_other,
                                                              const int32_t *__restrict__ t_off,
                                                              const int32_t *__restrict__ t_ref,
                                                              const int32_t *__restrict__ tri,
                                                              const uint8_t *__restrict__ fixed) {
    const int v = blockIdx.x * kRelaxThreads + threadIdx.x;
    if (v >= nv) return;
    const double2 xv = xin[v];
    if (fixed[v]) {
        xout[v] = xv;
        return;
    }
    double fx = 0.0, fy = 0.0;
    // edge springs: k_e (l - a0) along the edge, toward the other end when stretched
    for (int r = e_off[v]; r < e_off[v + 1]; ++r) {
        const double2 xo = xin[e_other[r]];
        const double dx = mi(xo.x - xv.x, G.Lx, G.periodic), dy = mi(xo.y - xv.y, G.Ly, G.periodic);
        const double ln = sqrt(dx * dx + dy * dy);
        const double f = G.k_e * (ln - G.a0) / ln;
        fx += f * dx;
        fy += f * dy;
    }
    // height springs of the incident triangles: -k_h (h - h0) dh/dx_v for each of the three
    // heights, h = (u x w)/|u| with u = b - a the base and w = c - a, c the apex
    for (int r = t_off[v]; r < t_off[v + 1]; ++r) {
        const int t = t_ref[r] >> 2, p = t_ref[r] & 3;
        double px[3], py[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 xk = xin[tri[3 * t + k]];
            px[k] = k == p ? 0.0 : mi(xk.x - xv.x, G.Lx, G.periodic);
            py[k] = k == p ? 0.0 : mi(xk.y - xv.y, G.Ly, G.periodic);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int a = (c + 1) % 3, b = (c + 2) % 3;
            const double ux = px[b] - px[a], uy = py[b] - py[a];
            const double wx = px[c] - px[a], wy = py[c] - py[a];
            const double lu = sqrt(ux * ux + uy * uy);
            const double h = (ux * wy - uy * wx) / lu;
            const double s = -G.k_h * (h - G.h0);
            const double dcx = -uy / lu, dcy = ux / lu;                       // perp(u)/|u|
            const double dbx = wy / lu - h * ux / (lu * lu);                  // -perp(w)/|u| - h u/|u|^2
            const double dby = -wx / lu - h * uy / (lu * lu);
            double gx, gy;
            if (p == c) {
                gx = dcx;
                gy = dcy;
            } else if (p == b) {
                gx = dbx;
                gy = dby;
            } else {
                gx = -(dbx + dcx);
                gy = -(dby + dcy);
            }
            fx += s * gx;
            fy += s * gy;
        }
    }
    double nx = xv.x + G.tau * fx, ny = xv.y + G.tau * fy;
    if (G.periodic) {
        nx = wrap(nx, G.Lx);
        ny = wrap(ny, G.Ly);
    }
    xout[v] = make_double2(nx, ny);
}

double mih(double d, double L, bool periodic) { return periodic ? d - L * std::nearbyint(d / L) : d; }

// Node -> edge (other end) and node -> triangle (triangle << 2 | local vertex) lists, each in
// ascending order of the other end / triangle.
void build_lists(int64_t nv, const std::vector<int32_t> &tri, std::vector<int32_t> &e_off,
                 std::vector<int32_t> &e_other, std::vector<int32_t> &t_off, std::vector<int32_t> &t_ref) {
    const int64_t nt = int64_t(tri.size()) / 3;
    std::vector<int64_t> keys;
    keys.reserve(6 * nt);
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q) {
            const int64_t a = tri[3 * j + q], b = tri[3 * j + (q + 1) % 3];
            keys.push_back(a * nv + b);  // both directions of every side
            keys.push_back(b * nv + a);
        }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    e_off.assign(nv + 1, 0);
    e_other.resize(keys.size());
    for (size_t k = 0; k < keys.size(); ++k) {
        ++e_off[keys[k] / nv + 1];
        e_other[k] = int32_t(keys[k] % nv);
    }
    for (int64_t v = 0; v < nv; ++v) e_off[v + 1] += e_off[v];
    t_off.assign(nv + 1, 0);
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q) ++t_off[tri[3 * j + q] + 1];
    for (int64_t v = 0; v < nv; ++v) t_off[v + 1] += t_off[v];
    t_ref.resize(3 * nt);
    std::vector<int32_t> fill(t_off.begin(), t_off.end() - 1);
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q) t_ref[fill[tri[3 * j + q]]++] = int32_t((j << 2) | q);
}

// Signed area x 2 of triangle j (minimum image, relative to its first vertex).
double twice_area(const std::vector<double> &xy, const std::vector<int32_t> &tri, int64_t j, bool periodic,
                  double Lx, double Ly) {
    const int32_t a = tri[3 * j], b = tri[3 * j + 1], c = tri[3 * j + 2];
    const double bx = mih(xy[2 * b] - xy[2 * a], Lx, periodic), by = mih(xy[2 * b + 1] - xy[2 * a + 1], Ly, periodic);
    const double cx = mih(xy[2 * c] - xy[2 * a], Lx, periodic), cy = mih(xy[2 * c + 1] - xy[2 * a + 1], Ly, periodic);
    return bx * cy - by * cx;
}

double spring_energy(const std::vector<double> &xy, const std::vector<int32_t> &tri, bool periodic, double Lx,
                     double Ly, double a0, double k_e, double k_h, int64_t nv) {
    const double h0 = a0 * std::sqrt(3.0) / 2.0;
    const int64_t nt = int64_t(tri.size()) / 3;
    std::vector<int64_t> keys;
    keys.reserve(3 * nt);
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q) {
            const int64_t a = tri[3 * j + q], b = tri[3 * j + (q + 1) % 3];
            keys.push_back(std::min(a, b) * nv + std::max(a, b));
        }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    double e = 0.0;
    for (int64_t k : keys) {
        const int64_t a = k / nv, b = k % nv;
        const double dx = mih(xy[2 * b] - xy[2 * a], Lx, periodic), dy = mih(xy[2 * b + 1] - xy[2 * a + 1], Ly, periodic);
        const double l = std::sqrt(dx * dx + dy * dy);
        e += 0.5 * k_e * (l - a0) * (l - a0);
    }
    for (int64_t j = 0; j < nt; ++j) {
        for (int c = 0; c < 3; ++c) {
            const int32_t va = tri[3 * j + (c + 1) % 3], vb = tri[3 * j + (c + 2) % 3], vc = tri[3 * j + c];
            const double ux = mih(xy[2 * vb] - xy[2 * va], Lx, periodic), uy = mih(xy[2 * vb + 1] - xy[2 * va + 1], Ly, periodic);
            const double wx = mih(xy[2 * vc] - xy[2 * va], Lx, periodic), wy = mih(xy[2 * vc + 1] - xy[2 * va + 1], Ly, periodic);
            const double h = (ux * wy - uy * wx) / std::sqrt(ux * ux + uy * uy);
            e += 0.5 * k_h * (h - h0) * (h - h0);
        }
    }
    return e;
}

template <typename T> int upload_host(DeviceBuffer &buf, const std::vector<T> &v, hipStream_t s) {
    int rc = buf.alloc(v.size() * sizeof(T));
    if (rc || v.empty()) return rc;
    TYEE_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return TYEE_OK;
}

// omega_max of (xy, tri) as a mesh of this domain, or +infinity when it is not a valid
// Delaunay mesh (a step of the relaxation may leave cocircular ties).
double omega_of(const std::vector<double> &xy, const std::vector<int32_t> &tri, const tyee_domain &dom) {
    Mesh m;
    if (build_mesh(xy.data(), int64_t(xy.size()) / 2, tri.data(), int64_t(tri.size()) / 3, dom, m) != TYEE_OK) {
        clear_error();
        return std::numeric_limits<double>::infinity();
    }
    double lam = 0.0;
    int64_t it = 0;
    const int rc = power_iteration(m, nullptr, 20000, 1e-12, 0, &lam, &it);
    clear_error();
    return rc == TYEE_OK || rc == TYEE_ENOTCONVERGED ? std::sqrt(lam) : std::numeric_limits<double>::infinity();
}

}  // namespace
}  // namespace tyee

using tyee::fail;

extern "C" int tyee_mesh_relax(const tyee_mesh *mesh, const tyee_relax_params *p, const int32_t *anchors,
                               int64_t n_anchors, void *stream, double *xy_out, int32_t *tri_out,
                               double *omega_rounds, tyee_relax_stats *stats) {
    using namespace tyee;
    if (!mesh || !p || !xy_out || !tri_out) return fail(TYEE_EINVAL, "null argument");
    if (p->rounds < 0 || p->iters < 0 || !(p->step > 0.0) || !(p->k_edge >= 0.0) || !(p->k_height >= 0.0) ||
        !(p->rest >= 0.0) || (n_anchors > 0 && !anchors) || n_anchors < 0)
        return fail(TYEE_EINVAL, "rounds, iters >= 0, step > 0, spring constants and rest length >= 0 required");
    const Mesh &m = mesh->m;
    const int64_t nv = m.nv, nt = m.nt;
    const bool periodic = m.periodic;
    if (nt >= (int64_t(1) << 29)) return fail(TYEE_EINVAL, "mesh too large for the relaxation's triangle ids");
    std::vector<uint8_t> fixed(nv, 0);
    for (int64_t v = 0; v < nv; ++v) fixed[v] = m.node_outer[v];  // outline of a closed resonator
    for (int64_t k = 0; k < n_anchors; ++k) {
        if (anchors[k] < 0 || anchors[k] >= nv) return fail(TYEE_EINVAL, "anchor out of range");
        fixed[anchors[k]] = 1;
    }
    tyee_domain dom{periodic ? TYEE_PERIODIC : TYEE_PEC_BOX, m.Lx, m.Ly, 0.0};
    RelaxGeom G{};
    G.periodic = periodic ? 1 : 0;
    G.Lx = m.Lx;
    G.Ly = m.Ly;
    G.a0 = p->rest > 0.0 ? p->rest : std::sqrt(4.0 * m.Lx * m.Ly / (std::sqrt(3.0) * double(nt)));
    G.h0 = G.a0 * std::sqrt(3.0) / 2.0;
    G.k_e = p->k_edge;
    G.k_h = p->k_height;
    G.tau = p->step;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<double> xy = m.xy;
    std::vector<int32_t> tri = m.tri;
    const double om0 = omega_of(xy, tri, dom);
    double best_om = om0;
    int32_t best_round = 0;
    std::vector<double> best_xy = xy;
    std::vector<int32_t> best_tri = tri;
    if (omega_rounds) omega_rounds[0] = om0;
    int64_t total_flips = 0;
    const double e0 = spring_energy(xy, tri, periodic, m.Lx, m.Ly, G.a0, G.k_e, G.k_h, nv);
    DeviceBuffer dx[2], d_eoff, d_eoth, d_toff, d_tref, d_tri, d_fixed;
    int rc = upload_host(d_fixed, fixed, s);
    if (!rc) rc = dx[0].alloc(size_t(nv) * sizeof(double2));
    if (!rc) rc = dx[1].alloc(size_t(nv) * sizeof(double2));
    if (rc) return rc;
    const int grid = int((nv + kRelaxThreads - 1) / kRelaxThreads);
    for (int32_t round = 1; round <= p->rounds; ++round) {
        std::vector<int32_t> e_off, e_other, t_off, t_ref;
        build_lists(nv, tri, e_off, e_other, t_off, t_ref);
        rc = upload_host(d_eoff, e_off, s);
        if (!rc) rc = upload_host(d_eoth, e_other, s);
        if (!rc) rc = upload_host(d_toff, t_off, s);
        if (!rc) rc = upload_host(d_tref, t_ref, s);
        if (!rc) rc = upload_host(d_tri, tri, s);
        if (rc) return rc;
        std::vector<double> moved(2 * nv);
        for (int attempt = 0;; ++attempt) {
            TYEE_HIP(hipMemcpyAsync(dx[0].p, xy.data(), size_t(nv) * sizeof(double2), hipMemcpyHostToDevice, s));
            int cur = 0;
            for (int32_t it = 0; it < p->iters; ++it) {
                k_relax_step<<<grid, kRelaxThreads, 0, s>>>(int(nv), G, dx[cur].as<double2>(), dx[1 - cur].as<double2>(),
                                                            d_eoff.as<int32_t>(), d_eoth.as<int32_t>(),
                                                            d_toff.as<int32_t>(), d_tref.as<int32_t>(),
                                                            d_tri.as<int32_t>(), d_fixed.as<uint8_t>());
                cur = 1 - cur;
            }
            TYEE_HIP(hipGetLastError());
            TYEE_HIP(hipMemcpyAsync(moved.data(), dx[cur].p, size_t(nv) * sizeof(double2), hipMemcpyDeviceToHost, s));
            TYEE_HIP(hipStreamSynchronize(s));
            bool folded = false;
            for (int64_t j = 0; j < nt && !folded; ++j)
                folded = !(twice_area(moved, tri, j, periodic, m.Lx, m.Ly) > 0.0);
            if (!folded) break;
            if (attempt == 5) return fail(TYEE_EUNSTABLE, "relaxation folds triangles even at a 32x smaller step");
            G.tau *= 0.5;  // a triangle turned over: redo the round with half the step
        }
        xy.swap(moved);
        int64_t fl = 0;
        rc = lawson_flip(xy, tri, periodic, m.Lx, m.Ly, nv, 50 * nt, &fl);
        if (rc) return rc;
        total_flips += fl;
        const double om = omega_of(xy, tri, dom);
        if (omega_rounds) omega_rounds[round] = om;
        if (!p->keep_best || om < best_om) {  // keep_best = 0: the last round is returned
            best_om = om;
            best_round = round;
            best_xy = xy;
            best_tri = tri;
        }
    }
    std::copy(best_xy.begin(), best_xy.end(), xy_out);
    std::copy(best_tri.begin(), best_tri.end(), tri_out);
    if (stats) {
        stats->omega_initial = om0;
        stats->omega_best = best_om;
        stats->best_round = best_round;
        stats->flips = total_flips;
        stats->energy_initial = e0;
        stats->energy_final = spring_energy(best_xy, best_tri, periodic, m.Lx, m.Ly, G.a0, G.k_e, G.k_h, nv);
        stats->step_used = G.tau;
    }
    return TYEE_OK;
}
