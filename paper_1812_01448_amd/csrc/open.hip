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
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
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
    int64_t ne_mesh = 0;                       // the triangle mesh's edges, ids 0 .. ne_mesh-1
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
    // edges: the mesh's ids (only its outer edges can be sides of a rectangle), then the
    // frame's by node pair
    std::map<std::pair<int32_t, int32_t>, int32_t> eid;
    for (int64_t i = 0; i < m.ne; ++i)
        if (!m.interior(i)) eid[{m.edge[2 * i], m.edge[2 * i + 1]}] = int32_t(i);
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
    f.ne_mesh = m.ne;
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

// The device holds each edge's line integral e_i = |e_i| E_i, so that a cell's update needs
// only the sign of each of its sides, carried in the sign of the stored edge id (id or ~id).
//
// E update: e_i = ca_i e_i + k_i (B_left - B_right), k_i = |e_i| dt / ((1 + sigma_i dt/2) d_i).
// The triangle mesh's edges lie in the box, where sigma is zero (ca = 1); only the frame's own
// edges (ids from nem up) read a decay factor.  A frame cell's B is the sum of its two parts.
// The frame's outer edges (one cell) keep their value.
template <typename T>
__global__ void k_open_edge(int32_t ne, int32_t nem, int32_t nt, const int2 *__restrict__ lr,
                            const T *__restrict__ k, const T *__restrict__ caf, const T *__restrict__ B,
                            const T *__restrict__ By, T *__restrict__ E) {
    const int i = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int2 c = lr[i];
    if (c.x < 0 || c.y < 0) return;
    const T bl = B[c.x] + (c.x >= nt ? By[c.x - nt] : T(0));
    const T br = B[c.y] + (c.y >= nt ? By[c.y - nt] : T(0));
    const T e = i >= nem ? caf[i - nem] * E[i] : E[i];
    E[i] = e + k[i] * (bl - br);
}

// s e_i for a signed id: id >= 0 reads +e_id, ~id reads -e_id.
template <typename T>
__device__ __forceinline__ T side(const T *__restrict__ E, int32_t id) {
    const T v = E[id ^ (id >> 31)];
    return id < 0 ? -v : v;
}

// B update.  Triangles (j < nt): B -= (dt/S) sum of s e over the three sides (ids t0, t1, t2).
// Frame cells: Bx = ax Bx - bx (left and right sides), By = ay By - by (bottom and top sides),
// fc = {ax, bx, ay, by} per cell with bx and by holding dt/S.
template <typename T>
__global__ void k_open_cell(int32_t ncell, int32_t nt, const int32_t *__restrict__ t0,
                            const int32_t *__restrict__ t1, const int32_t *__restrict__ t2,
                            const T *__restrict__ g, const int4 *__restrict__ fe, const T *__restrict__ fc,
                            const T *__restrict__ E, T *__restrict__ B, T *__restrict__ By) {
    const int j = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (j >= ncell) return;
    if (j < nt) {
        const T c = side(E, t0[j]) + side(E, t1[j]) + side(E, t2[j]);
        B[j] = B[j] - g[j] * c;
    } else {
        const int f = j - nt;
        const int4 q = fe[f];
        const T ax = fc[4 * f], bx = fc[4 * f + 1], ay = fc[4 * f + 2], by = fc[4 * f + 3];
        B[j] = ax * B[j] - bx * (side(E, q.x) + side(E, q.y));
        By[f] = ay * By[f] - by * (side(E, q.z) + side(E, q.w));
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
    // state: E (line integrals), B (triangles' B, frame cells' Bx), By (frame cells)
    tyee::DeviceBuffer E, B, By;
    // E update: lr, k per edge, caf per frame edge; B update: t0, t1, t2, g per triangle, fe, fc
    // per frame cell
    tyee::DeviceBuffer lr, k, caf, t0, t1, t2, g, fe, fc;
    int32_t graph_steps = 8;          // steps per captured graph (0: eager launches)
    hipGraphExec_t graph = nullptr;
    bool timing = false;
    std::vector<hipEvent_t> ev;   // timing: three events per step of a chunk of steps
    double ms_edge = 0.0, ms_cell = 0.0;
    int64_t timed = 0;
    // Fused stepping (tyee_open_set_fusion): the box's triangles are advanced by the fused
    // K-step kernel of a triangle-mesh simulation `box` (Morton numbering), and a band (the
    // frame plus the triangles within 2K + 3 rings of the box's sides) by K single steps of the
    // kernels above on its own compact arrays; see launch_open_fused.
    int fuse_K = 0;                   // 0: off
    std::unique_ptr<tyee_sim> box;
    int64_t bnbe = 0, bnbt = 0, bne = 0, bncell = 0, nw_e = 0, nw_t = 0;
    tyee::DeviceBuffer bE, bB, bBy, blr, bk, bt0, bt1, bt2, bg, bfe;   // band state and tables
    tyee::DeviceBuffer slot_e, slot_t;        // canonical box edge / triangle -> box device slot
    tyee::DeviceBuffer g_e, g_t;              // band box edge / triangle -> box device slot
    tyee::DeviceBuffer w_from_e, w_to_e, w_from_t, w_to_t;   // band cells written back to the box
    hipGraphExec_t fgraph = nullptr;  // kFusedGraphGroups fused groups, captured once
    hipStream_t side = nullptr;       // the band's branch inside the captured graph
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    ~tyee_open() {
        if (fgraph) (void)hipGraphExecDestroy(fgraph);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
        if (graph) (void)hipGraphExecDestroy(graph);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace tyee {
namespace {

int32_t signed_id(int32_t i, bool positive) { return positive ? i : ~i; }

template <typename T>
int upload_open(tyee_open &o) {
    const Frame &f = o.f;
    const double dt = o.dt;
    const size_t ts = sizeof(T);
    const int64_t nem = f.ne_mesh, nfe = f.ne - f.ne_mesh;
    std::vector<int2> lr(f.ne);
    std::vector<T> k(f.ne), caf(nfe);
    for (int64_t i = 0; i < f.ne; ++i) {
        lr[i] = make_int2(f.left[i], f.right[i]);
        const double s = 0.5 * f.sigma_e[i] * dt;
        if (i < nem && s != 0.0) return fail(TYEE_EINVAL, "a damped edge inside the box");
        if (i >= nem) caf[i - nem] = T((1.0 - s) / (1.0 + s));
        k[i] = f.left[i] >= 0 && f.right[i] >= 0 ? T(f.elen[i] * dt / (1.0 + s) / f.d[i]) : T(0);
    }
    std::vector<int32_t> t0(f.nt), t1(f.nt), t2(f.nt);
    std::vector<T> g(f.nt);
    std::vector<int4> fe(f.nf);
    std::vector<T> fc(4 * f.nf);
    for (int64_t j = 0; j < f.ncell; ++j) {
        const int32_t *e = &f.cell_edge[4 * j];
        int32_t id[4];
        for (int q = 0; q < 4; ++q) id[q] = e[q] >= 0 ? signed_id(e[q], f.cell_sl[4 * j + q] > 0.0) : 0;
        if (j < f.nt) {
            t0[j] = id[0];
            t1[j] = id[1];
            t2[j] = id[2];
            g[j] = T(dt / f.S[j]);
        } else {
            const int64_t q = j - f.nt;
            fe[q] = make_int4(id[0], id[1], id[2], id[3]);
            const double sx = 0.5 * f.sigma_x[j] * dt, sy = 0.5 * f.sigma_y[j] * dt;
            fc[4 * q] = T((1.0 - sx) / (1.0 + sx));
            fc[4 * q + 1] = T(dt / (1.0 + sx) / f.S[j]);
            fc[4 * q + 2] = T((1.0 - sy) / (1.0 + sy));
            fc[4 * q + 3] = T(dt / (1.0 + sy) / f.S[j]);
        }
    }
    auto put = [&](DeviceBuffer &b, const void *src, size_t bytes) -> int {
        int r = b.alloc(std::max<size_t>(bytes, 16));
        if (r) return r;
        if (src) TYEE_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, o.stream));
        else TYEE_HIP(hipMemsetAsync(b.p, 0, bytes, o.stream));
        return TYEE_OK;
    };
    int rc = 0;
    if ((rc = put(o.E, nullptr, f.ne * ts)) || (rc = put(o.B, nullptr, f.ncell * ts)) ||
        (rc = put(o.By, nullptr, f.nf * ts)) || (rc = put(o.lr, lr.data(), f.ne * sizeof(int2))) ||
        (rc = put(o.k, k.data(), f.ne * ts)) || (rc = put(o.caf, caf.data(), nfe * ts)) ||
        (rc = put(o.t0, t0.data(), f.nt * 4)) || (rc = put(o.t1, t1.data(), f.nt * 4)) ||
        (rc = put(o.t2, t2.data(), f.nt * 4)) || (rc = put(o.g, g.data(), f.nt * ts)) ||
        (rc = put(o.fe, fe.data(), f.nf * sizeof(int4))) || (rc = put(o.fc, fc.data(), 4 * f.nf * ts)))
        return rc;
    TYEE_HIP(hipStreamSynchronize(o.stream));
    return TYEE_OK;
}

template <typename T>
void enqueue_edge(tyee_open &o) {
    const int32_t ne = int32_t(o.f.ne);
    hipLaunchKernelGGL(k_open_edge<T>, dim3(unsigned(blocks_for(ne))), dim3(kBlock), 0, o.stream, ne,
                       int32_t(o.f.ne_mesh), int32_t(o.f.nt), o.lr.as<int2>(), o.k.as<T>(), o.caf.as<T>(),
                       o.B.as<T>(), o.By.as<T>(), o.E.as<T>());
}

template <typename T>
void enqueue_cell(tyee_open &o) {
    const int32_t nc = int32_t(o.f.ncell);
    hipLaunchKernelGGL(k_open_cell<T>, dim3(unsigned(blocks_for(nc))), dim3(kBlock), 0, o.stream, nc,
                       int32_t(o.f.nt), o.t0.as<int32_t>(), o.t1.as<int32_t>(), o.t2.as<int32_t>(), o.g.as<T>(),
                       o.fe.as<int4>(), o.fc.as<T>(), o.E.as<T>(), o.B.as<T>(), o.By.as<T>());
}

constexpr int64_t kTimedChunk = 256;   // steps whose events are recorded before any is read

// Per-launch HIP events around each E and B update (eager launches).
template <typename T>
int launch_timed(tyee_open &o, int64_t nsteps) {
    if (o.ev.empty()) {
        o.ev.assign(3 * kTimedChunk, nullptr);
        for (hipEvent_t &e : o.ev) TYEE_HIP(hipEventCreate(&e));
    }
    for (int64_t s0 = 0; s0 < nsteps; s0 += kTimedChunk) {
        const int64_t chunk = std::min(kTimedChunk, nsteps - s0);
        for (int64_t s = 0; s < chunk; ++s) {
            TYEE_HIP(hipEventRecord(o.ev[3 * s], o.stream));
            enqueue_edge<T>(o);
            TYEE_HIP(hipGetLastError());
            TYEE_HIP(hipEventRecord(o.ev[3 * s + 1], o.stream));
            enqueue_cell<T>(o);
            TYEE_HIP(hipGetLastError());
            TYEE_HIP(hipEventRecord(o.ev[3 * s + 2], o.stream));
        }
        TYEE_HIP(hipEventSynchronize(o.ev[3 * (chunk - 1) + 2]));
        for (int64_t s = 0; s < chunk; ++s) {
            float a = 0.0f, b = 0.0f;
            TYEE_HIP(hipEventElapsedTime(&a, o.ev[3 * s], o.ev[3 * s + 1]));
            TYEE_HIP(hipEventElapsedTime(&b, o.ev[3 * s + 1], o.ev[3 * s + 2]));
            o.ms_edge += a;
            o.ms_cell += b;
        }
        o.timed += chunk;
    }
    return TYEE_OK;
}

// Whole graphs of graph_steps steps (captured once: the buffers never move), the rest eager.
template <typename T>
int launch_open(tyee_open &o, int64_t nsteps) {
    if (o.timing) return launch_timed<T>(o, nsteps);
    int64_t done = 0;
    if (o.graph_steps > 0 && nsteps >= o.graph_steps) {
        if (!o.graph) {
            TYEE_HIP(hipStreamBeginCapture(o.stream, hipStreamCaptureModeThreadLocal));
            for (int32_t s = 0; s < o.graph_steps; ++s) {
                enqueue_edge<T>(o);
                enqueue_cell<T>(o);
            }
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(o.stream, &graph);
            if (e != hipSuccess) return fail(TYEE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&o.graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                o.graph = nullptr;
                return fail(TYEE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
        }
        for (; nsteps - done >= o.graph_steps; done += o.graph_steps) TYEE_HIP(hipGraphLaunch(o.graph, o.stream));
    }
    for (; done < nsteps; ++done) {
        enqueue_edge<T>(o);
        enqueue_cell<T>(o);
    }
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

// dst[to[i]] = src[from[i]] (a null map is the identity), i < n.
template <typename T>
__global__ void k_open_move(int32_t n, const int32_t *__restrict__ from, const int32_t *__restrict__ to,
                            const T *__restrict__ src, T *__restrict__ dst) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    dst[to ? to[i] : i] = src[from ? from[i] : i];
}

// Two such moves in one launch (i < max(n1, n2)).
template <typename T>
__global__ void k_open_move2(int32_t n1, const int32_t *__restrict__ f1, const int32_t *__restrict__ t1,
                             const T *__restrict__ s1, T *__restrict__ d1, int32_t n2, const int32_t *__restrict__ f2,
                             const int32_t *__restrict__ t2, const T *__restrict__ s2, T *__restrict__ d2) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n1) d1[t1 ? t1[i] : i] = s1[f1 ? f1[i] : i];
    if (i < n2) d2[t2 ? t2[i] : i] = s2[f2 ? f2[i] : i];
}

template <typename T>
void move2(hipStream_t st, int64_t n1, const DeviceBuffer *f1, const DeviceBuffer *t1, const T *s1, T *d1, int64_t n2,
           const DeviceBuffer *f2, const DeviceBuffer *t2, const T *s2, T *d2) {
    const int64_t n = std::max(n1, n2);
    if (n <= 0) return;
    auto ix = [](const DeviceBuffer *b) { return b ? b->as<int32_t>() : nullptr; };
    hipLaunchKernelGGL(k_open_move2<T>, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, int32_t(n1),
                       ix(f1), ix(t1), s1, d1, int32_t(n2), ix(f2), ix(t2), s2, d2);
}

template <typename T>
void move(hipStream_t st, int64_t n, const DeviceBuffer *from, const DeviceBuffer *to, const T *src, T *dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_open_move<T>, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, int32_t(n),
                       from ? from->as<int32_t>() : nullptr, to ? to->as<int32_t>() : nullptr, src, dst);
}

// The band and its tables.  A box triangle's ring is its distance, in triangles, from the box's
// sides (ring 1 touches a side).  The fused kernel holds the sides' edges fixed, so after K
// steps it is exact on the triangles of ring > K and on the edges between them; the band
// (every frame cell and edge, the triangles of ring <= 2K + 3 and their edges) advanced from
// the same state by K single steps, its inner cut held fixed, is exact on ring <= K + 3.  The
// band's triangles of ring <= K + 2 and the edges whose triangles all have ring <= K + 2 are
// written over the fused result.  Band numbering follows the mixed mesh's layout: box edges,
// then every frame edge in order; box triangles, then every frame cell in order.
int build_open_fusion(tyee_open &o, const Mesh &mesh, int K, int tile) {
    const Frame &f = o.f;
    if (mesh.nt != f.nt || mesh.ne != f.ne_mesh || mesh.nv > f.nv)
        return fail(TYEE_EINVAL, "the mesh is not the one the open boundary was built from");
    for (int64_t i = 0; i < mesh.ne; ++i)
        if (mesh.edge[2 * i] != f.edge[2 * i] || mesh.edge[2 * i + 1] != f.edge[2 * i + 1])
            return fail(TYEE_EINVAL, "the mesh is not the one the open boundary was built from");
    std::unique_ptr<tyee_mesh> copy(new tyee_mesh());
    copy->m = mesh;
    int rc = reorder_mesh(copy->m, TYEE_ORDER_MORTON, 0);
    tyee_sim *raw = nullptr;
    if (!rc) rc = tyee_sim_create(copy.get(), o.f64 ? TYEE_F64 : TYEE_F32, o.dt, o.stream, &raw);
    if (rc) return rc;
    std::unique_ptr<tyee_sim> box(raw);
    copy.reset();
    Sim &s = box->s;
    s.fusion = K;
    s.tile_tris = tile;
    if ((rc = build_tiling(s, K, tile))) return rc;
    // rings from the box's sides
    const int32_t far = 2 * K + 3, keep = K + 2;
    std::vector<int32_t> ring(mesh.nt, INT32_MAX), front;
    for (int64_t i = 0; i < mesh.ne; ++i)
        if (!mesh.interior(i)) {
            const int32_t j = mesh.R[i] >= 0 ? mesh.R[i] : mesh.L[i];
            if (j >= 0 && ring[j] > 1) {
                ring[j] = 1;
                front.push_back(j);
            }
        }
    for (int32_t r = 1; r < far && !front.empty(); ++r) {
        std::vector<int32_t> next;
        for (int32_t j : front)
            for (int q = 0; q < 3; ++q) {
                const int32_t i = mesh.A[3 * j + q];
                const int32_t o2 = mesh.R[i] == j ? mesh.L[i] : mesh.R[i];
                if (o2 >= 0 && ring[o2] == INT32_MAX) {
                    ring[o2] = r + 1;
                    next.push_back(o2);
                }
            }
        front.swap(next);
    }
    std::vector<int32_t> tloc(mesh.nt, -1), eloc(mesh.ne, -1), btri, bedge;
    for (int64_t j = 0; j < mesh.nt; ++j)
        if (ring[j] <= far) {
            tloc[j] = int32_t(btri.size());
            btri.push_back(int32_t(j));
        }
    for (int32_t j : btri)
        for (int q = 0; q < 3; ++q) eloc[mesh.A[3 * j + q]] = 0;
    for (int64_t i = 0; i < mesh.ne; ++i)
        if (eloc[i] == 0) {
            eloc[i] = int32_t(bedge.size());
            bedge.push_back(int32_t(i));
        }
    const int64_t nem = f.ne_mesh, nfe = f.ne - nem;
    o.bnbe = int64_t(bedge.size());
    o.bnbt = int64_t(btri.size());
    o.bne = o.bnbe + nfe;
    o.bncell = o.bnbt + f.nf;
    auto cell_of = [&](int32_t c) -> int32_t {   // mixed-mesh cell -> band cell (-1: not in the band)
        if (c < 0) return -1;
        return c < f.nt ? tloc[c] : int32_t(o.bnbt + (c - f.nt));
    };
    auto edge_of = [&](int32_t i) -> int32_t {   // mixed-mesh edge -> band edge (-1: not in the band)
        if (i < 0 || i >= f.ne) return -1;
        return i < nem ? eloc[i] : int32_t(o.bnbe + (i - nem));
    };
    const double dt = o.dt;
    std::vector<int2> lr(o.bne);
    std::vector<double> kk(o.bne);
    for (int64_t l = 0; l < o.bne; ++l) {
        const int64_t i = l < o.bnbe ? bedge[l] : nem + (l - o.bnbe);
        lr[l] = make_int2(cell_of(f.left[i]), cell_of(f.right[i]));
        const double sg = 0.5 * f.sigma_e[i] * dt;
        kk[l] = f.left[i] >= 0 && f.right[i] >= 0 ? f.elen[i] * dt / (1.0 + sg) / f.d[i] : 0.0;
    }
    std::vector<int32_t> t0(o.bnbt), t1(o.bnbt), t2(o.bnbt);
    std::vector<double> gg(o.bnbt);
    for (int64_t l = 0; l < o.bnbt; ++l) {
        const int64_t j = btri[l];
        int32_t id[3];
        for (int q = 0; q < 3; ++q) {
            const int32_t e = edge_of(f.cell_edge[4 * j + q]);
            if (e < 0) return fail(TYEE_EINVAL, "internal: a band triangle's edge is not in the band");
            id[q] = signed_id(e, f.cell_sl[4 * j + q] > 0.0);
        }
        t0[l] = id[0];
        t1[l] = id[1];
        t2[l] = id[2];
        gg[l] = dt / f.S[j];
    }
    std::vector<int4> fe(f.nf);
    for (int64_t q = 0; q < f.nf; ++q) {
        const int64_t j = f.nt + q;
        int32_t id[4];
        for (int c = 0; c < 4; ++c) {
            const int32_t e = edge_of(f.cell_edge[4 * j + c]);
            if (e < 0) return fail(TYEE_EINVAL, "internal: a frame cell's edge is not in the band");
            id[c] = signed_id(e, f.cell_sl[4 * j + c] > 0.0);
        }
        fe[q] = make_int4(id[0], id[1], id[2], id[3]);
    }
    // device slots of the box simulation, gathers and write-back pairs
    std::vector<int32_t> ge(o.bnbe), gt(o.bnbt), wfe, wte, wft, wtt;
    for (int64_t l = 0; l < o.bnbe; ++l) ge[l] = s.slot_e[bedge[l]];
    for (int64_t l = 0; l < o.bnbt; ++l) gt[l] = s.slot_t[btri[l]];
    for (int64_t l = 0; l < o.bnbt; ++l)
        if (ring[btri[l]] <= keep) {
            wft.push_back(int32_t(l));
            wtt.push_back(gt[l]);
        }
    for (int64_t l = 0; l < o.bnbe; ++l) {
        const int32_t i = bedge[l], a = mesh.R[i], b = mesh.L[i];
        if ((a < 0 || ring[a] <= keep) && (b < 0 || ring[b] <= keep)) {
            wfe.push_back(int32_t(l));
            wte.push_back(ge[l]);
        }
    }
    // host-side bounds checks of every index the kernels read
    for (const int2 &c : lr)
        if (c.x >= o.bncell || c.y >= o.bncell) return fail(TYEE_EINVAL, "internal: band cell out of range");
    for (int32_t v : ge)
        if (v < 0 || v >= s.ne) return fail(TYEE_EINVAL, "internal: box edge slot out of range");
    for (int32_t v : gt)
        if (v < 0 || v >= s.nt) return fail(TYEE_EINVAL, "internal: box triangle slot out of range");
    auto put = [&](DeviceBuffer &b, const void *src, size_t bytes) -> int {
        int r = b.alloc(std::max<size_t>(bytes, 16));
        if (r) return r;
        TYEE_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, o.stream));
        return TYEE_OK;
    };
    const size_t ts = o.f64 ? 8 : 4;
    std::vector<float> kf(kk.begin(), kk.end()), gf(gg.begin(), gg.end());
    const void *kp = o.f64 ? static_cast<const void *>(kk.data()) : static_cast<const void *>(kf.data());
    const void *gp = o.f64 ? static_cast<const void *>(gg.data()) : static_cast<const void *>(gf.data());
    if ((rc = o.bE.alloc(std::max<size_t>(o.bne * ts, 16))) || (rc = o.bB.alloc(std::max<size_t>(o.bncell * ts, 16))) ||
        (rc = o.bBy.alloc(std::max<size_t>(f.nf * ts, 16))) || (rc = put(o.blr, lr.data(), lr.size() * sizeof(int2))) ||
        (rc = put(o.bk, kp, o.bne * ts)) || (rc = put(o.bt0, t0.data(), t0.size() * 4)) ||
        (rc = put(o.bt1, t1.data(), t1.size() * 4)) || (rc = put(o.bt2, t2.data(), t2.size() * 4)) ||
        (rc = put(o.bg, gp, o.bnbt * ts)) || (rc = put(o.bfe, fe.data(), fe.size() * sizeof(int4))) ||
        (rc = put(o.slot_e, s.slot_e.data(), s.slot_e.size() * 4)) ||
        (rc = put(o.slot_t, s.slot_t.data(), s.slot_t.size() * 4)) || (rc = put(o.g_e, ge.data(), ge.size() * 4)) ||
        (rc = put(o.g_t, gt.data(), gt.size() * 4)) || (rc = put(o.w_from_e, wfe.data(), wfe.size() * 4)) ||
        (rc = put(o.w_to_e, wte.data(), wte.size() * 4)) || (rc = put(o.w_from_t, wft.data(), wft.size() * 4)) ||
        (rc = put(o.w_to_t, wtt.data(), wtt.size() * 4)))
        return rc;
    if (!o.side) TYEE_HIP(hipStreamCreateWithFlags(&o.side, hipStreamNonBlocking));
    if (!o.ev_fork) TYEE_HIP(hipEventCreateWithFlags(&o.ev_fork, hipEventDisableTiming));
    if (!o.ev_join) TYEE_HIP(hipEventCreateWithFlags(&o.ev_join, hipEventDisableTiming));
    TYEE_HIP(hipStreamSynchronize(o.stream));
    o.nw_e = int64_t(wfe.size());
    o.nw_t = int64_t(wft.size());
    o.box = std::move(box);
    o.fuse_K = K;
    return TYEE_OK;
}

template <typename T>
void enqueue_band(tyee_open &o, hipStream_t st) {
    hipLaunchKernelGGL(k_open_edge<T>, dim3(unsigned(blocks_for(o.bne))), dim3(kBlock), 0, st, int32_t(o.bne),
                       int32_t(o.bnbe), int32_t(o.bnbt), o.blr.as<int2>(), o.bk.as<T>(), o.caf.as<T>(), o.bB.as<T>(),
                       o.bBy.as<T>(), o.bE.as<T>());
    hipLaunchKernelGGL(k_open_cell<T>, dim3(unsigned(blocks_for(o.bncell))), dim3(kBlock), 0, st,
                       int32_t(o.bncell), int32_t(o.bnbt), o.bt0.as<int32_t>(), o.bt1.as<int32_t>(),
                       o.bt2.as<int32_t>(), o.bg.as<T>(), o.bfe.as<int4>(), o.fc.as<T>(), o.bE.as<T>(), o.bB.as<T>(),
                       o.bBy.as<T>());
}

// One fused group of K steps: the band gathers its box cells, one fused launch advances the
// box, K single steps the band, and the band's exact cells are written over the box's.
// With `side` (graph capture), the band's K steps run on the side stream beside the fused
// launch (they touch only the band's arrays, the fused launch only the box's), joined before
// the write-back; without it everything runs in order on the handle's stream.
template <typename T>
int enqueue_fused_group(tyee_open &o, bool side) {
    Sim &s = o.box->s;
    const hipStream_t st = o.stream;
    move2<T>(st, o.bnbe, &o.g_e, nullptr, s.Et().as<T>(), o.bE.as<T>(), o.bnbt, &o.g_t, nullptr, s.B().as<T>(),
             o.bB.as<T>());
    if (side) {
        TYEE_HIP(hipEventRecord(o.ev_fork, st));
        TYEE_HIP(hipStreamWaitEvent(o.side, o.ev_fork, 0));
        for (int k = 0; k < o.fuse_K; ++k) enqueue_band<T>(o, o.side);
        TYEE_HIP(hipEventRecord(o.ev_join, o.side));
    }
    int rc = launch_fused<T>(s, o.fuse_K);
    if (rc) return rc;
    if (side) TYEE_HIP(hipStreamWaitEvent(st, o.ev_join, 0));
    else
        for (int k = 0; k < o.fuse_K; ++k) enqueue_band<T>(o, st);
    move2<T>(st, o.nw_e, &o.w_from_e, &o.w_to_e, o.bE.as<T>(), s.Et().as<T>(), o.nw_t, &o.w_from_t, &o.w_to_t,
             o.bB.as<T>(), s.B().as<T>());
    return TYEE_OK;
}

constexpr int kFusedGraphGroups = 8;   // fused groups per captured graph (even: the box's two
                                       // field buffers are back in place after a replay)

// Fused stepping: the state moves into the box simulation and the band, whole groups of K
// steps run (replayed from a graph of kFusedGraphGroups groups unless graphs are off), and the
// state moves back; the rest of the steps run one launch per half-step.
template <typename T>
int launch_open_fused(tyee_open &o, int64_t nsteps) {
    const int K = o.fuse_K;
    const Frame &f = o.f;
    Sim &s = o.box->s;
    const hipStream_t st = o.stream;
    const int64_t cycles = nsteps / K, nem = f.ne_mesh, nfe = f.ne - nem;
    if (cycles > 0) {
        move<T>(st, nem, nullptr, &o.slot_e, o.E.as<T>(), s.Et().as<T>());
        move<T>(st, f.nt, nullptr, &o.slot_t, o.B.as<T>(), s.B().as<T>());
        move<T>(st, nfe, nullptr, nullptr, o.E.as<T>() + nem, o.bE.as<T>() + o.bnbe);
        move<T>(st, f.nf, nullptr, nullptr, o.B.as<T>() + f.nt, o.bB.as<T>() + o.bnbt);
        move<T>(st, f.nf, nullptr, nullptr, o.By.as<T>(), o.bBy.as<T>());
        int64_t c = 0;
        if (o.graph_steps > 0 && cycles >= kFusedGraphGroups) {
            if (!o.fgraph) {
                TYEE_HIP(hipGetLastError());
                TYEE_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                int rc = TYEE_OK;
                for (int g = 0; g < kFusedGraphGroups && !rc; ++g) rc = enqueue_fused_group<T>(o, true);
                hipGraph_t graph = nullptr;
                hipError_t e = hipStreamEndCapture(st, &graph);
                if (rc) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return rc;
                }
                if (e != hipSuccess) return fail(TYEE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
                e = hipGraphInstantiate(&o.fgraph, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    o.fgraph = nullptr;
                    return fail(TYEE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
                }
            }
            for (; cycles - c >= kFusedGraphGroups; c += kFusedGraphGroups) TYEE_HIP(hipGraphLaunch(o.fgraph, st));
        }
        for (; c < cycles; ++c) {
            int rc = enqueue_fused_group<T>(o, false);
            if (rc) return rc;
        }
        move<T>(st, nem, &o.slot_e, nullptr, s.Et().as<T>(), o.E.as<T>());
        move<T>(st, f.nt, &o.slot_t, nullptr, s.B().as<T>(), o.B.as<T>());
        move<T>(st, nfe, nullptr, nullptr, o.bE.as<T>() + o.bnbe, o.E.as<T>() + nem);
        move<T>(st, f.nf, nullptr, nullptr, o.bB.as<T>() + o.bnbt, o.B.as<T>() + f.nt);
        move<T>(st, f.nf, nullptr, nullptr, o.bBy.as<T>(), o.By.as<T>());
        TYEE_HIP(hipGetLastError());
    }
    const int64_t rest = nsteps - cycles * K;
    for (int64_t k = 0; k < rest; ++k) {
        enqueue_edge<T>(o);
        enqueue_cell<T>(o);
    }
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

// sqrt-free largest eigenvalue of K = -L_E L_B on the mixed mesh (undamped), FP64 power
// iteration on the host in the S-weighted inner product.
int open_power(const Frame &f, int64_t max_iter, double rtol, uint64_t seed, double *lambda, int64_t *iters) {
    std::vector<double> x(f.ncell), y(f.ncell), g(f.ne);
    for (int64_t j = 0; j < f.ncell; ++j) x[j] = 2.0 * (double(splitmix64(seed + uint64_t(j)) >> 11) * 0x1.0p-53) - 1.0;
    double lam = 0.0;
    int64_t it = 1;
    constexpr int64_t kChunks = 256;
    std::vector<double> part(3 * kChunks);
    for (; it <= max_iter; ++it) {
        // g = L_B x (per inner edge), y = -L_E g; per-chunk sums added in chunk order
        parallel_for(f.ne, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i)
                g[i] = f.left[i] >= 0 && f.right[i] >= 0 ? (x[f.left[i]] - x[f.right[i]]) / f.d[i] : 0.0;
        });
        parallel_for(kChunks, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                double sxy = 0.0, sxx = 0.0, syy = 0.0;
                for (int64_t j = f.ncell * c / kChunks; j < f.ncell * (c + 1) / kChunks; ++j) {
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
                part[3 * c] = sxy;
                part[3 * c + 1] = sxx;
                part[3 * c + 2] = syy;
            }
        }, f.ncell);
        double sxy = 0.0, sxx = 0.0, syy = 0.0;
        for (int64_t c = 0; c < kChunks; ++c) {
            sxy += part[3 * c];
            sxx += part[3 * c + 1];
            syy += part[3 * c + 2];
        }
        const double next = sxy / sxx;
        const double nrm = std::sqrt(syy);
        if (!(nrm > 0.0)) break;
        parallel_for(f.ncell, [&](int64_t j0, int64_t j1) {
            for (int64_t j = j0; j < j1; ++j) x[j] = y[j] / nrm;
        });
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
    // E is held as the line integral |e| E
    const bool line = field == TYEE_OPEN_E;
    TYEE_HIP(hipStreamSynchronize(o->stream));
    if (o->f64) {
        std::vector<double> tmp(values + off, values + off + n);
        if (line)
            for (int64_t i = 0; i < n; ++i) tmp[i] *= o->f.elen[i];
        TYEE_HIP(hipMemcpy(b->p, tmp.data(), size_t(n) * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(n);
        for (int64_t i = 0; i < n; ++i) tmp[i] = float(line ? values[off + i] * o->f.elen[i] : values[off + i]);
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
    const bool line = field == TYEE_OPEN_E;
    TYEE_HIP(hipStreamSynchronize(o->stream));
    if (field == TYEE_OPEN_BY) std::fill(values, values + o->f.nt, 0.0);
    if (o->f64) {
        TYEE_HIP(hipMemcpy(values + off, b->p, size_t(n) * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(n);
        TYEE_HIP(hipMemcpy(tmp.data(), b->p, size_t(n) * 4, hipMemcpyDeviceToHost));
        std::copy(tmp.begin(), tmp.end(), values + off);
    }
    if (line)
        for (int64_t i = 0; i < n; ++i) values[off + i] /= o->f.elen[i];
    return TYEE_OK;
}

extern "C" int tyee_open_step(tyee_open *o, int64_t nsteps) {
    using namespace tyee;
    if (!o || nsteps < 0) return fail(TYEE_EINVAL, "null handle or negative step count");
    if (o->fuse_K > 1 && !o->timing)
        return o->f64 ? launch_open_fused<double>(*o, nsteps) : launch_open_fused<float>(*o, nsteps);
    return o->f64 ? launch_open<double>(*o, nsteps) : launch_open<float>(*o, nsteps);
}

extern "C" int tyee_open_set_fusion(tyee_open *o, const tyee_mesh *mesh, int32_t steps_per_launch,
                                    int32_t tile_tris) {
    using namespace tyee;
    if (!o) return fail(TYEE_EINVAL, "null argument");
    // default depth: 7 in FP32 (open1415: 18.1 us per step against 19.5 at 6, 19.8 at 8, 20.9 at
    // 4: deeper groups spread the band's gather and write-back over more steps), 4 in FP64
    int K = steps_per_launch == 0 ? (o->f64 ? 4 : 7) : steps_per_launch;
    if (K < 1 || K > kMaxFusion) return fail(TYEE_EINVAL, "steps per launch must be 0 (default) or 1..8");
    if (tile_tris != 0 && (tile_tris < 256 || tile_tris > 8192))
        return fail(TYEE_EINVAL, "tile size must be 0 or in [256, 8192] triangles");
    if (hipStreamSynchronize(o->stream) != hipSuccess) return fail(TYEE_EDEVICE, "hipStreamSynchronize failed");
    if (o->fgraph) {
        (void)hipGraphExecDestroy(o->fgraph);
        o->fgraph = nullptr;
    }
    o->fuse_K = 0;
    o->box.reset();
    if (K == 1) return TYEE_OK;
    if (!mesh) return fail(TYEE_EINVAL, "null mesh");
    try {
        return build_open_fusion(*o, mesh->m, K, tile_tris);
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

extern "C" int tyee_open_set_graph(tyee_open *o, int32_t steps) {
    if (!o) return tyee::fail(TYEE_EINVAL, "null argument");
    if (steps < 0 || steps > 1024) return tyee::fail(TYEE_EINVAL, "steps per graph must be in 0 .. 1024");
    if (o->graph || o->fgraph) {
        if (hipStreamSynchronize(o->stream) != hipSuccess) return tyee::fail(TYEE_EDEVICE, "hipStreamSynchronize failed");
        if (o->graph) (void)hipGraphExecDestroy(o->graph);
        if (o->fgraph) (void)hipGraphExecDestroy(o->fgraph);
        o->graph = nullptr;
        o->fgraph = nullptr;
    }
    o->graph_steps = steps;
    return TYEE_OK;
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
