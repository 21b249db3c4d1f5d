// Tetrahedral mesh builder and power iteration (host, FP64) for the three-dimensional form of
// the scheme: E along the edges, B normal to the faces, the dual the Voronoi diagram of the
// nodes (the circumcentres of the tetrahedra), as the circumcentres of the triangles are in two
// dimensions.  Faraday's law on a face and Ampere's law on an edge's Voronoi polygon give
//   A_f  dB_f/dt = -sum over the face's edges of s |e| E_e,
//   A*_e dE_e/dt =  sum over the faces around the edge of s d_f B_f,
// with d_f the distance between the circumcentres on either side of face f along its normal,
// A*_e the area of the Voronoi polygon of edge e, s = +1 where the face's circuit runs along
// the edge.  A*_e is built face by face: the polygon's part between the two circumcentres on
// either side of face f is a triangle with base d_f and height h, the distance in the face's
// plane from the edge to the face's circumcentre (the 3-D form of d = hR + hL).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <memory>
#include <new>

#include "tet.hpp"

namespace tyee {
namespace {

struct V3 {
    double x, y, z;
};
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline V3 node(const std::vector<double> &xyz, int64_t v) { return {xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2]}; }

// a + (|u|^2 (v x w) + |v|^2 (w x u) + |w|^2 (u x v)) / (2 u . (v x w)), u = b - a, ...
V3 sphere_centre(V3 a, V3 b, V3 c, V3 d) {
    const V3 u = b - a, v = c - a, w = d - a;
    const V3 vw = cross(v, w), wu = cross(w, u), uv = cross(u, v);
    const double den = 2.0 * dot(u, vw);
    return a + (vw * dot(u, u) + wu * dot(v, v) + uv * dot(w, w)) * (1.0 / den);
}

// a + (|u|^2 (v x N) + |v|^2 (N x u)) / (2 |N|^2), N = u x v: the circumcentre in the plane
V3 circle_centre(V3 a, V3 b, V3 c) {
    const V3 u = b - a, v = c - a, N = cross(u, v);
    return a + (cross(v, N) * dot(u, u) + cross(N, u) * dot(v, v)) * (1.0 / (2.0 * dot(N, N)));
}

struct FaceRef {
    int32_t b, c, t, opp;
};

}  // namespace

int build_tet(const double *xyz, int64_t nv, const int32_t *tets, int64_t nt, TetMesh &m) {
    if (!xyz || !tets) return fail(TYEE_EINVAL, "null argument");
    if (nv < 4 || nt < 1) return fail(TYEE_EINVAL, "a tetrahedral mesh needs at least 4 nodes and 1 tetrahedron");
    if (nv >= (int64_t(1) << 31) || nt >= (int64_t(1) << 28))
        return fail(TYEE_EINVAL, "at most 2^31 - 1 nodes and 2^28 - 1 tetrahedra");
    m = TetMesh();
    m.nv = nv;
    m.nt = nt;
    m.xyz.assign(xyz, xyz + 3 * nv);
    m.tet.assign(tets, tets + 4 * nt);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t *q = &m.tet[4 * t];
        for (int k = 0; k < 4; ++k)
            if (q[k] < 0 || q[k] >= nv) return fail(TYEE_EINVAL, "a node index is out of range");
        const V3 a = node(m.xyz, q[0]);
        const double vol6 = dot(cross(node(m.xyz, q[1]) - a, node(m.xyz, q[2]) - a), node(m.xyz, q[3]) - a);
        if (!(std::fabs(vol6) > 0.0)) return fail(TYEE_EDEGENERATE, "a tetrahedron has no volume");
        if (vol6 < 0.0) std::swap(q[1], q[2]);
    }

    // edges: the six node pairs of every tetrahedron, bucketed by the lower node
    static const int kPair[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    std::vector<int64_t> start(nv + 1, 0);
    for (int64_t t = 0; t < nt; ++t)
        for (const auto &p : kPair) ++start[std::min(m.tet[4 * t + p[0]], m.tet[4 * t + p[1]]) + 1];
    for (int64_t v = 0; v < nv; ++v) start[v + 1] += start[v];
    std::vector<int32_t> higher(6 * nt);
    {
        std::vector<int64_t> pos(start.begin(), start.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (const auto &p : kPair) {
                const int32_t a = m.tet[4 * t + p[0]], b = m.tet[4 * t + p[1]];
                higher[pos[std::min(a, b)]++] = std::max(a, b);
            }
    }
    std::vector<int64_t> distinct(nv);
    parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            auto first = higher.begin() + start[v], last = higher.begin() + start[v + 1];
            std::sort(first, last);
            distinct[v] = std::unique(first, last) - first;
        }
    }, 6 * nt);
    std::vector<int64_t> eoff(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) eoff[v + 1] = eoff[v] + distinct[v];
    m.ne = eoff[nv];
    if (m.ne >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "the mesh has 2^31 edges or more");
    m.edge.resize(2 * m.ne);
    parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v)
            for (int64_t k = 0; k < distinct[v]; ++k) {
                m.edge[2 * (eoff[v] + k)] = int32_t(v);
                m.edge[2 * (eoff[v] + k) + 1] = higher[start[v] + k];
            }
    }, m.ne);
    auto edge_id = [&](int32_t a, int32_t b) -> int32_t {
        const int32_t lo = std::min(a, b), hi = std::max(a, b);
        auto first = higher.begin() + start[lo], last = first + distinct[lo];
        return int32_t(eoff[lo] + (std::lower_bound(first, last, hi) - first));
    };

    // faces: the four node triples of every tetrahedron, bucketed by the lowest node
    std::vector<int64_t> fstart(nv + 1, 0);
    auto sorted3 = [](int32_t p, int32_t q, int32_t r, int32_t out[3]) {
        if (p > q) std::swap(p, q);
        if (q > r) std::swap(q, r);
        if (p > q) std::swap(p, q);
        out[0] = p;
        out[1] = q;
        out[2] = r;
    };
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 4; ++k) {
            int32_t s[3], w = 0;
            const int32_t *q = &m.tet[4 * t];
            int32_t rest[3];
            for (int j = 0; j < 4; ++j)
                if (j != k) rest[w++] = q[j];
            sorted3(rest[0], rest[1], rest[2], s);
            ++fstart[s[0] + 1];
        }
    for (int64_t v = 0; v < nv; ++v) fstart[v + 1] += fstart[v];
    std::vector<FaceRef> refs(4 * nt);
    {
        std::vector<int64_t> pos(fstart.begin(), fstart.end() - 1);
        for (int64_t t = 0; t < nt; ++t)
            for (int k = 0; k < 4; ++k) {
                int32_t s[3], rest[3], w = 0;
                const int32_t *q = &m.tet[4 * t];
                for (int j = 0; j < 4; ++j)
                    if (j != k) rest[w++] = q[j];
                sorted3(rest[0], rest[1], rest[2], s);
                refs[pos[s[0]]++] = {s[1], s[2], int32_t(t), q[k]};
            }
    }
    std::vector<int64_t> fdistinct(nv);
    std::atomic<int> bad{0};
    parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            auto first = refs.begin() + fstart[v], last = refs.begin() + fstart[v + 1];
            std::sort(first, last, [](const FaceRef &x, const FaceRef &y) {
                return x.b < y.b || (x.b == y.b && (x.c < y.c || (x.c == y.c && x.t < y.t)));
            });
            int64_t n = 0;
            for (auto it = first; it != last;) {
                auto nx = it + 1;
                while (nx != last && nx->b == it->b && nx->c == it->c) ++nx;
                if (nx - it > 2) bad.store(1);
                ++n;
                it = nx;
            }
            fdistinct[v] = n;
        }
    }, 4 * nt);
    if (bad.load()) return fail(TYEE_ENONMANIFOLD, "a face is shared by more than two tetrahedra");
    std::vector<int64_t> foff(nv + 1, 0);
    for (int64_t v = 0; v < nv; ++v) foff[v + 1] = foff[v] + fdistinct[v];
    m.nf = foff[nv];
    if (m.nf >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "the mesh has 2^31 faces or more");
    m.face.resize(3 * m.nf);
    m.front.assign(m.nf, -1);
    m.back.assign(m.nf, -1);
    m.normal.resize(3 * m.nf);
    m.farea.resize(m.nf);
    parallel_for(nv, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            int64_t f = foff[v];
            auto first = refs.begin() + fstart[v], last = refs.begin() + fstart[v + 1];
            for (auto it = first; it != last; ++f) {
                const V3 a = node(m.xyz, v), b = node(m.xyz, it->b), c = node(m.xyz, it->c);
                const V3 N = cross(b - a, c - a);
                const double len = std::sqrt(dot(N, N));
                m.face[3 * f] = int32_t(v);
                m.face[3 * f + 1] = it->b;
                m.face[3 * f + 2] = it->c;
                m.farea[f] = 0.5 * len;
                m.normal[3 * f] = N.x / len;
                m.normal[3 * f + 1] = N.y / len;
                m.normal[3 * f + 2] = N.z / len;
                auto nx = it;
                for (; nx != last && nx->b == it->b && nx->c == it->c; ++nx) {
                    const double side = dot(node(m.xyz, nx->opp) - a, N);
                    int32_t &slot = side > 0.0 ? m.front[f] : m.back[f];
                    if (slot >= 0) bad.store(2);
                    slot = nx->t;
                }
                it = nx;
            }
        }
    }, 4 * nt);
    if (bad.load()) return fail(TYEE_ENONMANIFOLD, "two tetrahedra lie on one side of a face");
    refs.clear();
    refs.shrink_to_fit();
    m.face_edge.resize(3 * m.nf);
    parallel_for(m.nf, [&](int64_t f0, int64_t f1) {
        for (int64_t f = f0; f < f1; ++f) {
            const int32_t a = m.face[3 * f], b = m.face[3 * f + 1], c = m.face[3 * f + 2];
            m.face_edge[3 * f] = edge_id(a, b);
            m.face_edge[3 * f + 1] = edge_id(b, c);
            m.face_edge[3 * f + 2] = edge_id(a, c);
        }
    });

    // conducting walls
    m.inner_face.assign(m.nf, 1);
    m.inner_edge.assign(m.ne, 1);
    for (int64_t f = 0; f < m.nf; ++f)
        if (m.front[f] < 0 || m.back[f] < 0) {
            m.inner_face[f] = 0;
            for (int q = 0; q < 3; ++q) m.inner_edge[m.face_edge[3 * f + q]] = 0;
        }
    m.n_inner_face = std::count(m.inner_face.begin(), m.inner_face.end(), uint8_t(1));
    m.n_inner_edge = std::count(m.inner_edge.begin(), m.inner_edge.end(), uint8_t(1));

    // geometry
    m.elen.resize(m.ne);
    parallel_for(m.ne, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const V3 t = node(m.xyz, m.edge[2 * i + 1]) - node(m.xyz, m.edge[2 * i]);
            m.elen[i] = std::sqrt(dot(t, t));
        }
    });
    m.C.resize(3 * nt);
    parallel_for(nt, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            const int32_t *q = &m.tet[4 * t];
            const V3 c = sphere_centre(node(m.xyz, q[0]), node(m.xyz, q[1]), node(m.xyz, q[2]), node(m.xyz, q[3]));
            m.C[3 * t] = c.x;
            m.C[3 * t + 1] = c.y;
            m.C[3 * t + 2] = c.z;
        }
    });
    m.d.assign(m.nf, 0.0);
    parallel_for(m.nf, [&](int64_t f0, int64_t f1) {
        for (int64_t f = f0; f < f1; ++f) {
            if (!m.inner_face[f]) continue;
            const V3 cf = node(m.C, m.front[f]), cb = node(m.C, m.back[f]), n = node(m.normal, f);
            m.d[f] = dot(cf - cb, n);
        }
    });
    for (int64_t f = 0; f < m.nf; ++f)
        if (m.inner_face[f] && !(m.d[f] > 0.0))
            return fail(TYEE_ENOTDELAUNAY, "the circumcentres across a face are not in order (d <= 0): not Delaunay");

    // inner edge -> faces around it, then the Voronoi polygon areas
    m.ef_off.assign(m.ne + 1, 0);
    for (int64_t f = 0; f < m.nf; ++f) {
        if (!m.inner_face[f]) continue;
        for (int q = 0; q < 3; ++q)
            if (m.inner_edge[m.face_edge[3 * f + q]]) ++m.ef_off[m.face_edge[3 * f + q] + 1];
    }
    for (int64_t i = 0; i < m.ne; ++i) m.ef_off[i + 1] += m.ef_off[i];
    if (m.ef_off[m.ne] >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "too many edge-face incidences");
    m.ef.resize(m.ef_off[m.ne]);
    {
        std::vector<int64_t> pos(m.ef_off.begin(), m.ef_off.end() - 1);
        for (int64_t f = 0; f < m.nf; ++f) {
            if (!m.inner_face[f]) continue;
            for (int q = 0; q < 3; ++q) {
                const int32_t i = m.face_edge[3 * f + q];
                if (m.inner_edge[i]) m.ef[pos[i]++] = q == 2 ? ~int32_t(f) : int32_t(f);
            }
        }
    }
    m.dual_area.assign(m.ne, 0.0);
    parallel_for(m.ne, [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            if (!m.inner_edge[i]) continue;
            const int32_t lo = m.edge[2 * i], hi = m.edge[2 * i + 1];
            const V3 p = node(m.xyz, lo), r = node(m.xyz, hi);
            const V3 t = (r - p) * (1.0 / m.elen[i]), mid = (p + r) * 0.5;
            double area = 0.0;
            for (int64_t k = m.ef_off[i]; k < m.ef_off[i + 1]; ++k) {
                const int32_t id = m.ef[k], f = id < 0 ? ~id : id;
                const int32_t *q = &m.face[3 * f];
                const int32_t w = q[0] != lo && q[0] != hi ? q[0] : (q[1] != lo && q[1] != hi ? q[1] : q[2]);
                const V3 cc = circle_centre(node(m.xyz, q[0]), node(m.xyz, q[1]), node(m.xyz, q[2]));
                V3 u = node(m.xyz, w) - p;
                u = u - t * dot(u, t);
                const double h = dot(cc - mid, u) / std::sqrt(dot(u, u));
                area += 0.5 * h * m.d[f];
            }
            m.dual_area[i] = area;
        }
    });
    for (int64_t i = 0; i < m.ne; ++i)
        if (m.inner_edge[i] && !(m.dual_area[i] > 0.0))
            return fail(TYEE_ENOTDELAUNAY, "an edge's Voronoi polygon has no positive area: not Delaunay");
    return TYEE_OK;
}

int tet_power(const TetMesh &m, int64_t max_iter, double rtol, uint64_t seed, double *lambda, int64_t *iters) {
    std::vector<double> x(m.ne, 0.0), y(m.ne), g(m.nf);
    for (int64_t i = 0; i < m.ne; ++i)
        if (m.inner_edge[i]) x[i] = 2.0 * (double(splitmix64(seed + uint64_t(i)) >> 11) * 0x1.0p-53) - 1.0;
    constexpr int64_t kChunks = 256;
    std::vector<double> part(3 * kChunks);
    double lam = 0.0;
    int64_t it = 1;
    for (; it <= max_iter; ++it) {
        // g = dB/dt of x on every inner face, y = -dE/dt of g on every inner edge: y = K x
        parallel_for(m.nf, [&](int64_t f0, int64_t f1) {
            for (int64_t f = f0; f < f1; ++f) {
                if (!m.inner_face[f]) {
                    g[f] = 0.0;
                    continue;
                }
                const int32_t *e = &m.face_edge[3 * f];
                g[f] = -(m.elen[e[0]] * x[e[0]] + m.elen[e[1]] * x[e[1]] - m.elen[e[2]] * x[e[2]]) / m.farea[f];
            }
        });
        parallel_for(kChunks, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                double sxy = 0.0, sxx = 0.0, syy = 0.0;
                for (int64_t i = m.ne * c / kChunks; i < m.ne * (c + 1) / kChunks; ++i) {
                    if (!m.inner_edge[i]) {
                        y[i] = 0.0;
                        continue;
                    }
                    double acc = 0.0;
                    for (int64_t k = m.ef_off[i]; k < m.ef_off[i + 1]; ++k) {
                        const int32_t id = m.ef[k], f = id < 0 ? ~id : id;
                        acc += (id < 0 ? -m.d[f] : m.d[f]) * g[f];
                    }
                    y[i] = -acc / m.dual_area[i];
                    const double w = m.dual_area[i] * m.elen[i];
                    sxy += w * x[i] * y[i];
                    sxx += w * x[i] * x[i];
                    syy += w * y[i] * y[i];
                }
                part[3 * c] = sxy;
                part[3 * c + 1] = sxx;
                part[3 * c + 2] = syy;
            }
        }, m.ne);
        double sxy = 0.0, sxx = 0.0, syy = 0.0;
        for (int64_t c = 0; c < kChunks; ++c) {
            sxy += part[3 * c];
            sxx += part[3 * c + 1];
            syy += part[3 * c + 2];
        }
        const double next = sxy / sxx, nrm = std::sqrt(syy);
        if (!(nrm > 0.0)) break;
        parallel_for(m.ne, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) x[i] = y[i] / nrm;
        });
        const bool done = it > 1 && std::fabs(next - lam) <= rtol * std::fabs(next);
        lam = next;
        if (done) break;
    }
    *lambda = lam;
    if (iters) *iters = std::min(it, max_iter);
    return it <= max_iter ? TYEE_OK : fail(TYEE_ENOTCONVERGED, "power iteration hit max_iter");
}

}  // namespace tyee

extern "C" int tyee_tet_create(const double *xyz, int64_t nv, const int32_t *tets, int64_t nt, tyee_tet **out) {
    using namespace tyee;
    if (!out) return fail(TYEE_EINVAL, "null argument");
    *out = nullptr;
    try {
        std::unique_ptr<tyee_tet> h(new tyee_tet());
        const int rc = build_tet(xyz, nv, tets, nt, h->m);
        if (rc) return rc;
        *out = h.release();
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

extern "C" int tyee_tet_sizes(const tyee_tet *m, int64_t out[7]) {
    if (!m || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    out[0] = m->m.nv;
    out[1] = m->m.ne;
    out[2] = m->m.nf;
    out[3] = m->m.nt;
    out[4] = m->m.n_inner_edge;
    out[5] = m->m.n_inner_face;
    out[6] = int64_t(m->m.ef.size());
    return TYEE_OK;
}

extern "C" int tyee_tet_view(const tyee_tet *m, int32_t *edge, int32_t *face, int32_t *face_edge, double *elen,
                             double *dual_area, double *farea, double *d, double *C) {
    if (!m) return tyee::fail(TYEE_EINVAL, "null argument");
    auto copy = [](auto *dst, const auto &src) {
        if (dst) std::copy(src.begin(), src.end(), dst);
    };
    copy(edge, m->m.edge);
    copy(face, m->m.face);
    copy(face_edge, m->m.face_edge);
    copy(elen, m->m.elen);
    copy(dual_area, m->m.dual_area);
    copy(farea, m->m.farea);
    copy(d, m->m.d);
    copy(C, m->m.C);
    return TYEE_OK;
}

extern "C" int tyee_tet_cfl(const tyee_tet *m, int64_t max_iter, double rtol, uint64_t seed, double *lambda,
                            int64_t *iters) {
    if (!m || !lambda) return tyee::fail(TYEE_EINVAL, "null argument");
    if (max_iter < 2 || !(rtol >= 0.0)) return tyee::fail(TYEE_EINVAL, "max_iter >= 2 and rtol >= 0 required");
    if (m->m.n_inner_edge == 0) return tyee::fail(TYEE_EINVAL, "the mesh has no inner edge");
    try {
        return tyee::tet_power(m->m, max_iter, rtol, seed, lambda, iters);
    } catch (const std::bad_alloc &) {
        return tyee::fail(TYEE_ENOMEM, "host allocation failed");
    }
}

extern "C" int tyee_tet_destroy(tyee_tet *m) {
    delete m;
    return TYEE_OK;
}
