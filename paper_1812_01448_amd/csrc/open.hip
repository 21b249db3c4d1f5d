// Open boundary: the triangle mesh of a closed box tied to a rectangular frame of PML layers
// (the paper's Conclusion: the scheme runs on mixed triangle and quad meshes, so a mesh with
// rectangular boundaries can be joined to a structured frame that carries PML layers).
//
// A rectangle's circumcentre is its centre, on the perpendicular bisector of every side as a
// triangle's circumcentre is, so eqs. 3-4 hold on the mixed mesh unchanged: E on every edge
// along its tangent (lower node id to higher), dE/dt = (B_left - B_right)/d with d the distance
// between the two centres across the edge; dB/dt = -(1/S) sum over the cell's edges of s |e| E
// (s = +1 where the edge runs counter-clockwise around the cell).  In the frame, B is split
// (Berenger): Bx takes the curl of the cell's two vertical edges and decays with sigma_x, By
// that of its two horizontal edges and decays with sigma_y; an edge parallel to x decays with
// sigma_y, one parallel to y with sigma_x; sigma(rho) = sigma_max (rho / depth)^grading with
// rho the distance beyond the box.  The frame's outer wall is a perfect conductor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <utility>
#include <vector>

#include "sim.hpp"

namespace tyee {
namespace {

// The mixed mesh on the host, in canonical numbering: the triangle mesh's nodes, edges and
// triangles keep their ids; the frame's new nodes follow ordered by (y, x), its edges follow
// the mesh's ordered by (lower, higher) node id, its rectangles follow the triangles ordered
// by the (y, x) of their centres.
struct Frame {
    int64_t nv = 0, ne = 0, ncell = 0, nt = 0, nf = 0, n_inner = 0;
    std::vector<double> xy;                    // [nv][2]
    std::vector<int32_t> edge;                 // [ne][2]
    std::vector<int32_t> left, right;          // [ne], -1 on the frame's outer wall
    std::vector<double> elen, d, sigma_e;      // [ne]
    std::vector<uint8_t> vertical;             // [ne]
    std::vector<double> S, O, sigma_x, sigma_y;  // [ncell] (O [ncell][2])
    std::vector<int32_t> cell_edge;            // [ncell][4]: a rectangle's vertical pair first; -1 pads
    std::vector<double> cell_sl;               // [ncell][4]: s |e|
};

double profile(double rho, const tyee_pml_params &p) {
    if (!(rho > 0.0)) return 0.0;
    const double depth = double(p.layers) * p.width;
    return p.sigma_max * std::pow(rho / depth, p.grading);
}

int build_frame(const Mesh &m, const tyee_pml_params &p, Frame &f) {
    if (m.periodic) return fail(TYEE_EINVAL, "the frame needs a closed box, not a torus");
    if (p.layers < 1 || p.layers > 4096 || !(p.width > 0.0) || !(p.sigma_max >= 0.0) || !(p.grading >= 0.0))
        return fail(TYEE_EINVAL, "pml: layers in 1 .. 4096, width > 0, sigma_max >= 0, grading >= 0");
    const double Lx = m.Lx, Ly = m.Ly, h = p.width;
    const int n = p.layers;
    // the mesh's nodes on the four sides of the box, and its outer edges all on them
    std::vector<int32_t> bottom, top, lside, rside;
    for (int64_t v = 0; v < m.nv; ++v) {
        if (!m.node_outer[v]) continue;
        const double x = m.xy[2 * v], y = m.xy[2 * v + 1];
        if (y == 0.0) bottom.push_back(int32_t(v));
        if (y == Ly) top.push_back(int32_t(v));
        if (x == 0.0) lside.push_back(int32_t(v));
        if (x == Lx) rside.push_back(int32_t(v));
    }
    auto by = [&](int k) {
        return [&m, k](int32_t a, int32_t b) { return m.xy[2 * a + k] < m.xy[2 * b + k]; };
    };
    std::sort(bottom.begin(), bottom.end(), by(0));
    std::sort(top.begin(), top.end(), by(0));
    std::sort(lside.begin(), lside.end(), by(1));
    std::sort(rside.begin(), rside.end(), by(1));
    for (int64_t i = 0; i < m.ne; ++i) {
        if (m.interior(i)) continue;
        const int32_t a = m.edge[2 * i], b = m.edge[2 * i + 1];
        const double ax = m.xy[2 * a], ay = m.xy[2 * a + 1], bx = m.xy[2 * b], byv = m.xy[2 * b + 1];
        const bool on = (ay == 0.0 && byv == 0.0) || (ay == Ly && byv == Ly) || (ax == 0.0 && bx == 0.0) ||
                        (ax == Lx && bx == Lx);
        if (!on) return fail(TYEE_EINVAL, "the mesh's outer edges must lie on the sides of the box [0, Lx] x [0, Ly]");
    }
    if (bottom.size() < 2 || top.size() < 2 || lside.size() < 2 || rside.size() < 2)
        return fail(TYEE_EINVAL, "the mesh has no nodes on a side of the box");
    // rectangles (x0, x1, y0, y1); the inner line of a strip is exactly the box side
    struct Rect {
        double x0, x1, y0, y1;
    };
    std::vector<Rect> rects;
    auto xb = [&](int32_t v) { return m.xy[2 * v]; };
    auto yb = [&](int32_t v) { return m.xy[2 * v + 1]; };
    for (int k = 0; k < n; ++k) {
        const double in_lo = k ? -double(k) * h : 0.0, out_lo = -double(k + 1) * h;
        const double in_hx = k ? Lx + double(k) * h : Lx, out_hx = Lx + double(k + 1) * h;
        const double in_hy = k ? Ly + double(k) * h : Ly, out_hy = Ly + double(k + 1) * h;
        for (size_t a = 0; a + 1 < bottom.size(); ++a) rects.push_back({xb(bottom[a]), xb(bottom[a + 1]), out_lo, in_lo});
        for (size_t a = 0; a + 1 < top.size(); ++a) rects.push_back({xb(top[a]), xb(top[a + 1]), in_hy, out_hy});
        for (size_t b = 0; b + 1 < lside.size(); ++b) rects.push_back({out_lo, in_lo, yb(lside[b]), yb(lside[b + 1])});
        for (size_t b = 0; b + 1 < rside.size(); ++b) rects.push_back({in_hx, out_hx, yb(rside[b]), yb(rside[b + 1])});
        for (int r = 0; r < n; ++r) {
            const double r_in_lo = r ? -double(r) * h : 0.0, r_out_lo = -double(r + 1) * h;
            const double r_in_hy = r ? Ly + double(r) * h : Ly, r_out_hy = Ly + double(r + 1) * h;
            rects.push_back({out_lo, in_lo, r_out_lo, r_in_lo});
            rects.push_back({out_lo, in_lo, r_in_hy, r_out_hy});
            rects.push_back({in_hx, out_hx, r_out_lo, r_in_lo});
            rects.push_back({in_hx, out_hx, r_in_hy, r_out_hy});
        }
    }
    // nodes
    std::map<std::pair<double, double>, int32_t> node;
    for (auto *s : {&bottom, &top, &lside, &rside})
        for (int32_t v : *s) node[{m.xy[2 * v], m.xy[2 * v + 1]}] = v;
    std::vector<std::pair<double, double>> fresh;
    for (const Rect &q : rects)
        for (auto pt : {std::make_pair(q.x0, q.y0), std::make_pair(q.x1, q.y0), std::make_pair(q.x1, q.y1),
                        std::make_pair(q.x0, q.y1)})
            if (!node.count(pt)) {
                node[pt] = -1;
                fresh.push_back(pt);
            }
    std::sort(fresh.begin(), fresh.end(), [](const auto &a, const auto &b) {
        return a.second < b.second || (a.second == b.second && a.first < b.first);
    });
    f.nv = m.nv + int64_t(fresh.size());
    f.xy.assign(m.xy.begin(), m.xy.end());
    for (size_t q = 0; q < fresh.size(); ++q) {
        node[fresh[q]] = int32_t(m.nv + int64_t(q));
        f.xy.push_back(fresh[q].first);
        f.xy.push_back(fresh[q].second);
    }
    std::sort(rects.begin(), rects.end(), [](const Rect &a, const Rect &b) {
        const double ay = 0.5 * (a.y0 + a.y1), by2 = 0.5 * (b.y0 + b.y1);
        const double ax = 0.5 * (a.x0 + a.x1), bx2 = 0.5 * (b.x0 + b.x1);
        return ay < by2 || (ay == by2 && ax < bx2);
    });
    f.nt = m.nt;
    f.nf = int64_t(rects.size());
    f.ncell = f.nt + f.nf;
    // edges: the mesh's ids, then the frame's by node pair
    std::map<std::pair<int32_t, int32_t>, int32_t> eid;
    for (int64_t i = 0; i < m.ne; ++i) eid[{m.edge[2 * i], m.edge[2 * i + 1]}] = int32_t(i);
    auto key = [](int32_t a, int32_t b) { return std::make_pair(std::min(a, b), std::max(a, b)); };
    std::vector<std::array<int32_t, 4>> corner(rects.size());
    std::set<std::pair<int32_t, int32_t>> fresh_edges;
    for (size_t c = 0; c < rects.size(); ++c) {
        const Rect &q = rects[c];
        corner[c] = {node[{q.x0, q.y0}], node[{q.x1, q.y0}], node[{q.x1, q.y1}], node[{q.x0, q.y1}]};
        for (int s = 0; s < 4; ++s) {
            auto k2 = key(corner[c][s], corner[c][(s + 1) % 4]);
            if (!eid.count(k2)) fresh_edges.insert(k2);
        }
    }
    f.ne = m.ne + int64_t(fresh_edges.size());
    f.edge.assign(m.edge.begin(), m.edge.end());
    {
        int32_t next = int32_t(m.ne);
        for (const auto &k2 : fresh_edges) {
            eid[k2] = next++;
            f.edge.push_back(k2.first);
            f.edge.push_back(k2.second);
        }
    }
    // cells: edges, centres, areas; a rectangle lists its left and right sides (vertical), then
    // its bottom and top sides
    f.cell_edge.assign(size_t(4) * f.ncell, -1);
    f.S.resize(f.ncell);
    f.O.resize(2 * f.ncell);
    std::vector<double> centroid(2 * f.ncell);
    for (int64_t j = 0; j < m.nt; ++j) {
        for (int q = 0; q < 3; ++q) f.cell_edge[4 * j + q] = m.A[3 * j + q];
        f.S[j] = m.S[j];
        f.O[2 * j] = m.O[2 * j];
        f.O[2 * j + 1] = m.O[2 * j + 1];
        double cx = 0.0, cy = 0.0;
        for (int q = 0; q < 3; ++q) {
            cx += m.xy[2 * m.tri[3 * j + q]];
            cy += m.xy[2 * m.tri[3 * j + q] + 1];
        }
        centroid[2 * j] = cx / 3.0;
        centroid[2 * j + 1] = cy / 3.0;
    }
    for (size_t c = 0; c < rects.size(); ++c) {
        const int64_t j = m.nt + int64_t(c);
        const auto &k = corner[c];
        f.cell_edge[4 * j + 0] = eid[key(k[3], k[0])];   // left side
        f.cell_edge[4 * j + 1] = eid[key(k[1], k[2])];   // right side
        f.cell_edge[4 * j + 2] = eid[key(k[0], k[1])];   // bottom
        f.cell_edge[4 * j + 3] = eid[key(k[2], k[3])];   // top
        const Rect &q = rects[c];
        f.S[j] = (q.x1 - q.x0) * (q.y1 - q.y0);
        f.O[2 * j] = centroid[2 * j] = 0.5 * (q.x0 + q.x1);
        f.O[2 * j + 1] = centroid[2 * j + 1] = 0.5 * (q.y0 + q.y1);
    }
    // edge geometry, left and right cells, damping
    f.left.assign(f.ne, -1);
    f.right.assign(f.ne, -1);
    f.elen.resize(f.ne);
    f.d.assign(f.ne, 0.0);
    f.vertical.resize(f.ne);
    f.sigma_e.resize(f.ne);
    auto rho = [](double v, double L) { return std::max(0.0, std::max(-v, v - L)); };
    for (int64_t i = 0; i < f.ne; ++i) {
        const int32_t a = f.edge[2 * i], b = f.edge[2 * i + 1];
        const double tx = f.xy[2 * b] - f.xy[2 * a], ty = f.xy[2 * b + 1] - f.xy[2 * a + 1];
        f.elen[i] = std::hypot(tx, ty);
        f.vertical[i] = std::fabs(tx) <= 1e-12 * f.elen[i];
        const double mx = 0.5 * (f.xy[2 * a] + f.xy[2 * b]), my = 0.5 * (f.xy[2 * a + 1] + f.xy[2 * b + 1]);
        f.sigma_e[i] = f.vertical[i] ? profile(rho(mx, Lx), p) : profile(rho(my, Ly), p);
    }
    for (int64_t j = 0; j < f.ncell; ++j)
        for (int q = 0; q < 4; ++q) {
            const int32_t i = f.cell_edge[4 * j + q];
            if (i < 0) continue;
            const int32_t a = f.edge[2 * i], b = f.edge[2 * i + 1];
            const double tx = f.xy[2 * b] - f.xy[2 * a], ty = f.xy[2 * b + 1] - f.xy[2 * a + 1];
            const double rx = centroid[2 * j] - f.xy[2 * a], ry = centroid[2 * j + 1] - f.xy[2 * a + 1];
            (tx * ry - ty * rx > 0.0 ? f.left[i] : f.right[i]) = int32_t(j);
        }
    f.cell_sl.assign(size_t(4) * f.ncell, 0.0);
    for (int64_t j = 0; j < f.ncell; ++j)
        for (int q = 0; q < 4; ++q) {
            const int32_t i = f.cell_edge[4 * j + q];
            if (i >= 0) f.cell_sl[4 * j + q] = (f.left[i] == j ? 1.0 : -1.0) * f.elen[i];
        }
    f.n_inner = 0;
    for (int64_t i = 0; i < f.ne; ++i) {
        if (f.left[i] < 0 || f.right[i] < 0) continue;
        ++f.n_inner;
        const int32_t a = f.edge[2 * i], b = f.edge[2 * i + 1];
        const double tx = f.xy[2 * b] - f.xy[2 * a], ty = f.xy[2 * b + 1] - f.xy[2 * a + 1];
        const double nx = -ty / f.elen[i], ny = tx / f.elen[i];   // towards the left cell
        const int32_t l = f.left[i], r = f.right[i];
        f.d[i] = (f.O[2 * l] - f.O[2 * r]) * nx + (f.O[2 * l + 1] - f.O[2 * r + 1]) * ny;
        if (!(f.d[i] > 0.0)) return fail(TYEE_ENOTDELAUNAY, "a centre-to-centre distance across an edge is not positive");
    }
    f.sigma_x.assign(f.ncell, 0.0);
    f.sigma_y.assign(f.ncell, 0.0);
    for (int64_t j = m.nt; j < f.ncell; ++j) {
        f.sigma_x[j] = profile(rho(f.O[2 * j], Lx), p);
        f.sigma_y[j] = profile(rho(f.O[2 * j + 1], Ly), p);
    }
    return TYEE_OK;
}

// E_i = ca_i E_i + cbd_i (B_left - B_right), B of a frame cell the sum of its two parts; the
// frame's outer edges (no second cell) stay at zero.
template <typename T>
__global__ void k_open_edge(int32_t ne, int32_t nt, const int2 *__restrict__ lr, const T *__restrict__ ca,
                            const T *__restrict__ cbd, const T *__restrict__ B, const T *__restrict__ By,
                            T *__restrict__ E) {
    const int i = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int2 c = lr[i];
    if (c.x < 0 || c.y < 0) return;
    const T bl = B[c.x] + (c.x >= nt ? By[c.x - nt] : T(0));
    const T br = B[c.y] + (c.y >= nt ? By[c.y - nt] : T(0));
    E[i] = ca[i] * E[i] + cbd[i] * (bl - br);
}

// Triangles: B -= (dt/S) sum_q s|e| E.  Frame cells: Bx = ax Bx - bx (its vertical sides' terms),
// By = ay By - by (its horizontal sides' terms), bx and by holding the 1/S.
template <typename T>
__global__ void k_open_cell(int32_t ncell, int32_t nt, const int4 *__restrict__ ce, const T *__restrict__ sl,
                            const T *__restrict__ ax, const T *__restrict__ bx, const T *__restrict__ ay,
                            const T *__restrict__ by, const T *__restrict__ E, T *__restrict__ B,
                            T *__restrict__ By) {
    const int j = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (j >= ncell) return;
    const int4 e = ce[j];
    const T c0 = sl[4 * j] * E[e.x], c1 = sl[4 * j + 1] * E[e.y], c2 = sl[4 * j + 2] * E[e.z];
    if (j < nt) {
        B[j] = B[j] - bx[j] * (c0 + c1 + c2);
    } else {
        const T c3 = sl[4 * j + 3] * E[e.w];
        B[j] = ax[j] * B[j] - bx[j] * (c0 + c1);
        const int f = j - nt;
        By[f] = ay[f] * By[f] - by[f] * (c2 + c3);
    }
}

}  // namespace
}  // namespace tyee

struct tyee_open {
    tyee::Frame f;
    bool f64 = false;
    double dt = 0.0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    tyee::DeviceBuffer E, B, By, lr, ca, cbd, ce, sl, ax, bx, ay, by;
    bool timing = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    double ms_edge = 0.0, ms_cell = 0.0;
    int64_t timed = 0;
    ~tyee_open() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace tyee {
namespace {

template <typename T>
int upload_open(tyee_open &o) {
    const Frame &f = o.f;
    const double dt = o.dt;
    const size_t ts = sizeof(T);
    std::vector<int2> lr(f.ne);
    std::vector<T> ca(f.ne), cbd(f.ne);
    for (int64_t i = 0; i < f.ne; ++i) {
        lr[i] = make_int2(f.left[i], f.right[i]);
        const double s = 0.5 * f.sigma_e[i] * dt;
        ca[i] = T((1.0 - s) / (1.0 + s));
        cbd[i] = f.left[i] >= 0 && f.right[i] >= 0 ? T(dt / (1.0 + s) / f.d[i]) : T(0);
    }
    std::vector<int4> ce(f.ncell);
    std::vector<T> sl(4 * f.ncell), ax(f.ncell), bx(f.ncell), ay(f.nf), by(f.nf);
    for (int64_t j = 0; j < f.ncell; ++j) {
        const int32_t *e = &f.cell_edge[4 * j];
        // a triangle's missing fourth side reads its first edge (a valid address, not used)
        ce[j] = make_int4(e[0], e[1], e[2], e[3] >= 0 ? e[3] : e[0]);
        for (int q = 0; q < 4; ++q) sl[4 * j + q] = T(f.cell_sl[4 * j + q]);
        const double sx = 0.5 * f.sigma_x[j] * dt;
        ax[j] = T((1.0 - sx) / (1.0 + sx));
        bx[j] = T(dt / (1.0 + sx) / f.S[j]);
        if (j >= f.nt) {
            const double sy = 0.5 * f.sigma_y[j] * dt;
            ay[j - f.nt] = T((1.0 - sy) / (1.0 + sy));
            by[j - f.nt] = T(dt / (1.0 + sy) / f.S[j]);
        }
    }
    int rc = 0;
    auto put = [&](DeviceBuffer &b, const void *src, size_t bytes) -> int {
        int r = b.alloc(std::max<size_t>(bytes, 16));
        if (r) return r;
        if (src) TYEE_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, o.stream));
        else TYEE_HIP(hipMemsetAsync(b.p, 0, bytes, o.stream));
        return TYEE_OK;
    };
    if ((rc = put(o.E, nullptr, f.ne * ts)) || (rc = put(o.B, nullptr, f.ncell * ts)) ||
        (rc = put(o.By, nullptr, f.nf * ts)) || (rc = put(o.lr, lr.data(), f.ne * sizeof(int2))) ||
        (rc = put(o.ca, ca.data(), f.ne * ts)) || (rc = put(o.cbd, cbd.data(), f.ne * ts)) ||
        (rc = put(o.ce, ce.data(), f.ncell * sizeof(int4))) || (rc = put(o.sl, sl.data(), 4 * f.ncell * ts)) ||
        (rc = put(o.ax, ax.data(), f.ncell * ts)) || (rc = put(o.bx, bx.data(), f.ncell * ts)) ||
        (rc = put(o.ay, ay.data(), f.nf * ts)) || (rc = put(o.by, by.data(), f.nf * ts)))
        return rc;
    TYEE_HIP(hipStreamSynchronize(o.stream));
    return TYEE_OK;
}

template <typename T>
int launch_open(tyee_open &o, int64_t nsteps) {
    const Frame &f = o.f;
    const int32_t ne = int32_t(f.ne), nc = int32_t(f.ncell), nt = int32_t(f.nt);
    const dim3 ge(unsigned((ne + kBlock - 1) / kBlock)), gc(unsigned((nc + kBlock - 1) / kBlock));
    for (int64_t s = 0; s < nsteps; ++s) {
        if (o.timing) TYEE_HIP(hipEventRecord(o.ev[0], o.stream));
        hipLaunchKernelGGL(k_open_edge<T>, ge, dim3(kBlock), 0, o.stream, ne, nt, o.lr.as<int2>(), o.ca.as<T>(),
                           o.cbd.as<T>(), o.B.as<T>(), o.By.as<T>(), o.E.as<T>());
        TYEE_HIP(hipGetLastError());
        if (o.timing) TYEE_HIP(hipEventRecord(o.ev[1], o.stream));
        hipLaunchKernelGGL(k_open_cell<T>, gc, dim3(kBlock), 0, o.stream, nc, nt, o.ce.as<int4>(), o.sl.as<T>(),
                           o.ax.as<T>(), o.bx.as<T>(), o.ay.as<T>(), o.by.as<T>(), o.E.as<T>(), o.B.as<T>(),
                           o.By.as<T>());
        TYEE_HIP(hipGetLastError());
        if (o.timing) {
            TYEE_HIP(hipEventRecord(o.ev[2], o.stream));
            TYEE_HIP(hipEventSynchronize(o.ev[2]));
            float a = 0.0f, b = 0.0f;
            TYEE_HIP(hipEventElapsedTime(&a, o.ev[0], o.ev[1]));
            TYEE_HIP(hipEventElapsedTime(&b, o.ev[1], o.ev[2]));
            o.ms_edge += a;
            o.ms_cell += b;
            ++o.timed;
        }
    }
    return TYEE_OK;
}

// sqrt-free largest eigenvalue of K = -L_E L_B on the mixed mesh (undamped), FP64 power
// iteration on the host in the S-weighted inner product.
int open_power(const Frame &f, int64_t max_iter, double rtol, uint64_t seed, double *lambda, int64_t *iters) {
    std::vector<double> x(f.ncell), y(f.ncell), g(f.ne);
    for (int64_t j = 0; j < f.ncell; ++j) x[j] = 2.0 * (double(splitmix64(seed + uint64_t(j)) >> 11) * 0x1.0p-53) - 1.0;
    double lam = 0.0;
    int64_t it = 1;
    for (; it <= max_iter; ++it) {
        // g = L_B x (per inner edge), y = -L_E g
        for (int64_t i = 0; i < f.ne; ++i)
            g[i] = f.left[i] >= 0 && f.right[i] >= 0 ? (x[f.left[i]] - x[f.right[i]]) / f.d[i] : 0.0;
        double sxy = 0.0, sxx = 0.0, syy = 0.0;
        for (int64_t j = 0; j < f.ncell; ++j) {
            double acc = 0.0;
            for (int q = 0; q < 4; ++q) {
                const int32_t i = f.cell_edge[4 * j + q];
                if (i >= 0) acc += f.cell_sl[4 * j + q] * g[i];
            }
            y[j] = acc / f.S[j];
            sxy += f.S[j] * x[j] * y[j];
            sxx += f.S[j] * x[j] * x[j];
            syy += f.S[j] * y[j] * y[j];
        }
        const double next = sxy / sxx;
        const double nrm = std::sqrt(syy);
        if (!(nrm > 0.0)) break;
        for (int64_t j = 0; j < f.ncell; ++j) x[j] = y[j] / nrm;
        const bool done = it > 1 && std::fabs(next - lam) <= rtol * std::fabs(next);
        lam = next;
        if (done) break;
    }
    *lambda = lam;
    if (iters) *iters = std::min(it, max_iter);
    return it <= max_iter ? TYEE_OK : fail(TYEE_ENOTCONVERGED, "power iteration hit max_iter");
}

}  // namespace
}  // namespace tyee

extern "C" int tyee_open_create(const tyee_mesh *mesh, const tyee_pml_params *pml, int32_t prec, double dt,
                                void *stream, tyee_open **out) {
    using namespace tyee;
    if (!mesh || !pml || !out) return fail(TYEE_EINVAL, "null argument");
    *out = nullptr;
    if (prec != TYEE_F32 && prec != TYEE_F64) return fail(TYEE_EINVAL, "prec must be TYEE_F32 or TYEE_F64");
    if (!(dt > 0.0)) return fail(TYEE_EINVAL, "dt must be positive");
    try {
        std::unique_ptr<tyee_open> o(new tyee_open());
        int rc = build_frame(mesh->m, *pml, o->f);
        if (rc) return rc;
        if (o->f.ne >= (int64_t(1) << 31) || o->f.ncell >= (int64_t(1) << 31))
            return fail(TYEE_EINVAL, "the mixed mesh has 2^31 edges or cells or more");
        o->f64 = prec == TYEE_F64;
        o->dt = dt;
        TYEE_HIP(hipGetDevice(&o->device));
        if (stream) {
            o->stream = static_cast<hipStream_t>(stream);
        } else {
            TYEE_HIP(hipStreamCreateWithFlags(&o->stream, hipStreamNonBlocking));
            o->own_stream = true;
        }
        for (hipEvent_t &e : o->ev) TYEE_HIP(hipEventCreate(&e));
        rc = o->f64 ? upload_open<double>(*o) : upload_open<float>(*o);
        if (rc) return rc;
        *out = o.release();
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

extern "C" int tyee_open_sizes(const tyee_open *o, int64_t out[5]) {
    if (!o || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    out[0] = o->f.nv;
    out[1] = o->f.ne;
    out[2] = o->f.ncell;
    out[3] = o->f.nf;
    out[4] = o->f.n_inner;
    return TYEE_OK;
}

extern "C" int tyee_open_frame(const tyee_mesh *mesh, const tyee_pml_params *pml, int64_t sizes[5], double *xy,
                               int32_t *edge, int32_t *cell_edge, double *elen, double *d, double *S, double *O,
                               double *sigma_e, double *sigma_x, double *sigma_y) {
    using namespace tyee;
    if (!mesh || !pml || !sizes) return fail(TYEE_EINVAL, "null argument");
    try {
        Frame f;
        const int rc = build_frame(mesh->m, *pml, f);
        if (rc) return rc;
        sizes[0] = f.nv;
        sizes[1] = f.ne;
        sizes[2] = f.ncell;
        sizes[3] = f.nf;
        sizes[4] = f.n_inner;
        auto copy = [](auto *dst, const auto &src) {
            if (dst) std::copy(src.begin(), src.end(), dst);
        };
        copy(xy, f.xy);
        copy(edge, f.edge);
        copy(cell_edge, f.cell_edge);
        copy(elen, f.elen);
        copy(d, f.d);
        copy(S, f.S);
        copy(O, f.O);
        copy(sigma_e, f.sigma_e);
        copy(sigma_x, f.sigma_x);
        copy(sigma_y, f.sigma_y);
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

extern "C" int tyee_open_cfl(const tyee_open *o, int64_t max_iter, double rtol, uint64_t seed, double *lambda,
                             int64_t *iters) {
    if (!o || !lambda) return tyee::fail(TYEE_EINVAL, "null argument");
    if (max_iter < 2 || !(rtol >= 0.0)) return tyee::fail(TYEE_EINVAL, "max_iter >= 2 and rtol >= 0 required");
    try {
        return tyee::open_power(o->f, max_iter, rtol, seed, lambda, iters);
    } catch (const std::bad_alloc &) {
        return tyee::fail(TYEE_ENOMEM, "host allocation failed");
    }
}

namespace {
int open_field(const tyee_open *o, int32_t field, int64_t *n, tyee::DeviceBuffer **buf, int64_t *off) {
    switch (field) {
    case TYEE_OPEN_E: *n = o->f.ne; *buf = const_cast<tyee::DeviceBuffer *>(&o->E); *off = 0; return TYEE_OK;
    case TYEE_OPEN_BX: *n = o->f.ncell; *buf = const_cast<tyee::DeviceBuffer *>(&o->B); *off = 0; return TYEE_OK;
    case TYEE_OPEN_BY: *n = o->f.nf; *buf = const_cast<tyee::DeviceBuffer *>(&o->By); *off = o->f.nt; return TYEE_OK;
    default: return tyee::fail(TYEE_EINVAL, "field must be TYEE_OPEN_E, TYEE_OPEN_BX or TYEE_OPEN_BY");
    }
}
}  // namespace

extern "C" int tyee_open_set_state(tyee_open *o, int32_t field, const double *values) {
    using namespace tyee;
    if (!o || !values) return fail(TYEE_EINVAL, "null argument");
    int64_t n = 0, off = 0;
    DeviceBuffer *b = nullptr;
    int rc = open_field(o, field, &n, &b, &off);
    if (rc) return rc;
    TYEE_HIP(hipStreamSynchronize(o->stream));
    if (o->f64) {
        TYEE_HIP(hipMemcpy(b->p, values + off, size_t(n) * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(values + off, values + off + n);
        TYEE_HIP(hipMemcpy(b->p, tmp.data(), size_t(n) * 4, hipMemcpyHostToDevice));
    }
    return TYEE_OK;
}

extern "C" int tyee_open_get_state(tyee_open *o, int32_t field, double *values) {
    using namespace tyee;
    if (!o || !values) return fail(TYEE_EINVAL, "null argument");
    int64_t n = 0, off = 0;
    DeviceBuffer *b = nullptr;
    int rc = open_field(o, field, &n, &b, &off);
    if (rc) return rc;
    TYEE_HIP(hipStreamSynchronize(o->stream));
    if (field == TYEE_OPEN_BY) std::fill(values, values + o->f.nt, 0.0);
    if (o->f64) {
        TYEE_HIP(hipMemcpy(values + off, b->p, size_t(n) * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(n);
        TYEE_HIP(hipMemcpy(tmp.data(), b->p, size_t(n) * 4, hipMemcpyDeviceToHost));
        std::copy(tmp.begin(), tmp.end(), values + off);
    }
    return TYEE_OK;
}

extern "C" int tyee_open_step(tyee_open *o, int64_t nsteps) {
    using namespace tyee;
    if (!o || nsteps < 0) return fail(TYEE_EINVAL, "null handle or negative step count");
    return o->f64 ? launch_open<double>(*o, nsteps) : launch_open<float>(*o, nsteps);
}

extern "C" int tyee_open_sync(tyee_open *o) {
    if (!o) return tyee::fail(TYEE_EINVAL, "null argument");
    if (hipStreamSynchronize(o->stream) != hipSuccess) return tyee::fail(TYEE_EDEVICE, "hipStreamSynchronize failed");
    return TYEE_OK;
}

extern "C" int tyee_open_set_timing(tyee_open *o, int32_t on) {
    if (!o) return tyee::fail(TYEE_EINVAL, "null argument");
    o->timing = on != 0;
    o->ms_edge = o->ms_cell = 0.0;
    o->timed = 0;
    return TYEE_OK;
}

extern "C" int tyee_open_kernel_ms(const tyee_open *o, double out[2], int64_t *steps) {
    if (!o || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    out[0] = o->ms_edge;
    out[1] = o->ms_cell;
    if (steps) *steps = o->timed;
    return TYEE_OK;
}

extern "C" int tyee_open_destroy(tyee_open *o) {
    delete o;
    return TYEE_OK;
}
