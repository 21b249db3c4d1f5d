// Host-side mesh preparation for libtyee: connectivity, FP64 geometry with the Delaunay
// (positive dual length) check, locality numbering and the omega_max iteration.
//
// Connectivity and geometry follow Fig. 2 and eqs. 3-4 of arXiv:1812.01448; the
// signed dual length d = hR + hL is the |O_R O_L| of eq. 3 and the weight of metric (7).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "internal.hpp"

namespace tyee {

namespace {
thread_local std::string g_last_error;

inline double min_image(double delta, double period, bool periodic) {
    return periodic ? delta - period * std::nearbyint(delta / period) : delta;
}
}  // namespace

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}
void clear_error() { g_last_error.clear(); }

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t work) {
    const int64_t chunks = 256;
    if ((work < 0 ? n : work) < 65536) {
        for (int64_t c = 0; c < chunks; ++c) fn(n * c / chunks, n * (c + 1) / chunks);
        return;
    }
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (int64_t c; (c = next.fetch_add(1)) < chunks;) fn(n * c / chunks, n * (c + 1) / chunks);
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nth; ++t) pool.emplace_back(worker);
    worker();
    for (auto &t : pool) t.join();
}

uint64_t splitmix64(uint64_t x) {
    // Steele, Lea, Flood: SplitMix64 output function for state x (after the gamma step)
    x += 0x9E3779B97F4A7C15ULL;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    return x ^ (x >> 31);
}

// Spread the 16 bits of v to the even bit positions (magic-mask bit spreading).
static inline uint32_t spread_bits16(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

uint32_t morton_key(uint32_t qx, uint32_t qz) { return spread_bits16(qx) | (spread_bits16(qz) << 1); }

// ---------------------------------------------------------------------------------------
// connectivity and geometry
// ---------------------------------------------------------------------------------------

int build_mesh(const double *xy, int64_t nv, const int32_t *tri, int64_t nt,
               const tyee_domain &dom, Mesh &m) {
    if (!xy || !tri || nv <= 0 || nt <= 0) return fail(TYEE_EINVAL, "empty or null mesh input");
    if (nv > INT32_MAX || 3 * nt > INT32_MAX) return fail(TYEE_EINVAL, "mesh too large for int32 ids");
    if (!(dom.Lx > 0.0) || !(dom.Ly > 0.0)) return fail(TYEE_EINVAL, "domain Lx, Ly must be > 0");
    if (dom.kind != TYEE_PEC_BOX && dom.kind != TYEE_PERIODIC) return fail(TYEE_EINVAL, "unknown domain kind");
    m = Mesh();
    m.nv = nv;
    m.nt = nt;
    m.periodic = dom.kind == TYEE_PERIODIC;
    m.Lx = dom.Lx;
    m.Ly = dom.Ly;
    m.xy.assign(xy, xy + 2 * nv);
    m.tri.assign(tri, tri + 3 * nt);
    for (int64_t k = 0; k < 3 * nt; ++k)
        if (m.tri[k] < 0 || m.tri[k] >= nv) return fail(TYEE_EINVAL, "triangle references a missing node");

    const bool per = m.periodic;
    auto rel = [&](int32_t from, int32_t to, double out[2]) {
        out[0] = min_image(m.xy[2 * to] - m.xy[2 * from], m.Lx, per);
        out[1] = min_image(m.xy[2 * to + 1] - m.xy[2 * from + 1], m.Ly, per);
    };

    // 1. counter-clockwise winding (swap v1, v2), reject degenerate triangles
    const double degenerate = 1e-14 * m.Lx * m.Ly;
    for (int64_t j = 0; j < nt; ++j) {
        int32_t *v = &m.tri[3 * j];
        double b[2], c[2];
        rel(v[0], v[1], b);
        rel(v[0], v[2], c);
        double twice_area = b[0] * c[1] - b[1] * c[0];
        if (std::fabs(twice_area) <= degenerate)
            return fail(TYEE_EDEGENERATE, "degenerate triangle " + std::to_string(j));
        if (twice_area < 0.0) std::swap(v[1], v[2]);
    }

    // 2. edges: bucket the directed sides by their lower node, then order each bucket by
    //    (upper node, side); walking the buckets in node order yields the lexicographic
    //    (lo, hi) numbering.
    std::vector<int64_t> start(nv + 1, 0);
    for (int64_t k = 0; k < 3 * nt; ++k) {
        int32_t a = m.tri[k], b = m.tri[k - k % 3 + (k % 3 + 1) % 3];
        ++start[std::min(a, b) + 1];
    }
    for (int64_t v = 0; v < nv; ++v) start[v + 1] += start[v];
    std::vector<std::pair<int32_t, int32_t>> bucket(3 * nt);  // (hi, side = 3 t + q)
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t k = 0; k < 3 * nt; ++k) {
            int32_t a = m.tri[k], b = m.tri[k - k % 3 + (k % 3 + 1) % 3];
            bucket[fill[std::min(a, b)]++] = {std::max(a, b), int32_t(k)};
        }
    }
    for (int64_t v = 0; v < nv; ++v) std::sort(bucket.begin() + start[v], bucket.begin() + start[v + 1]);

    m.A.assign(3 * nt, -1);
    m.edge.reserve(3 * nt / 2 + 4);
    m.R.reserve(3 * nt / 2 + 4);
    m.L.reserve(3 * nt / 2 + 4);
    for (int64_t v = 0; v < nv; ++v) {
        for (int64_t k = start[v]; k < start[v + 1];) {
            int64_t g = k;
            while (g < start[v + 1] && bucket[g].first == bucket[k].first) ++g;
            const int32_t id = int32_t(m.edge.size() / 2);
            int32_t r = -1, l = -1;
            if (g - k > 2) return fail(TYEE_ENONMANIFOLD, "edge shared by more than two triangles");
            for (int64_t s = k; s < g; ++s) {
                int32_t side = bucket[s].second, t = side / 3, q = side % 3;
                bool forward = m.tri[side] == int32_t(v);  // side runs lo -> hi
                int32_t &slot = forward ? r : l;
                if (slot >= 0) return fail(TYEE_ENONMANIFOLD, "edge used twice in one direction");
                slot = t;
                m.A[3 * t + q] = id;
            }
            if (g - k == 1) {
                if (per) return fail(TYEE_EPERIODIC, "periodic mesh has an unmatched edge");
                ++m.nb;
            }
            m.edge.push_back(int32_t(v));
            m.edge.push_back(bucket[k].first);
            m.R.push_back(r);
            m.L.push_back(l);
            k = g;
        }
    }
    m.ne = int64_t(m.R.size());
    m.sgn.resize(3 * nt);
    for (int64_t k = 0; k < 3 * nt; ++k) m.sgn[k] = m.R[m.A[k]] == int32_t(k / 3) ? 1 : -1;

    // 3. edge vectors, lengths, midpoints
    const int64_t ne = m.ne;
    m.evec.resize(2 * ne);
    m.elen.resize(ne);
    m.C.resize(2 * ne);
    m.node_outer.assign(nv, 0);
    for (int64_t i = 0; i < ne; ++i) {
        int32_t lo = m.edge[2 * i], hi = m.edge[2 * i + 1];
        double e[2];
        rel(lo, hi, e);
        m.evec[2 * i] = e[0];
        m.evec[2 * i + 1] = e[1];
        m.elen[i] = std::hypot(e[0], e[1]);
        m.C[2 * i] = m.xy[2 * lo] + e[0] / 2.0;
        m.C[2 * i + 1] = m.xy[2 * lo + 1] + e[1] / 2.0;
        if (!m.interior(i)) m.node_outer[lo] = m.node_outer[hi] = 1;
    }

    // 4. per-triangle frame (origin at vertex 0): area, circumcentre, half dual lengths
    m.S.resize(nt);
    m.O.resize(2 * nt);
    m.hR.assign(ne, 0.0);
    m.hL.assign(ne, 0.0);
    for (int64_t j = 0; j < nt; ++j) {
        const int32_t *v = &m.tri[3 * j];
        double P[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        rel(v[0], v[1], P[1]);
        rel(v[0], v[2], P[2]);
        const double *b = P[1], *c = P[2];
        double twice_area = b[0] * c[1] - b[1] * c[0];
        double den = 2.0 * twice_area;
        double bb = b[0] * b[0] + b[1] * b[1], cc = c[0] * c[0] + c[1] * c[1];
        double ux = (c[1] * bb - b[1] * cc) / den;
        double uz = (b[0] * cc - c[0] * bb) / den;
        m.S[j] = twice_area / 2.0;
        m.O[2 * j] = m.xy[2 * v[0]] + ux;
        m.O[2 * j + 1] = m.xy[2 * v[0] + 1] + uz;
        for (int q = 0; q < 3; ++q) {
            const int32_t i = m.A[3 * j + q];
            const double tx = m.evec[2 * i] / m.elen[i], tz = m.evec[2 * i + 1] / m.elen[i];
            const double nx = -tz, nz = tx;  // left normal of e_i
            const bool is_r = m.sgn[3 * j + q] > 0;
            const double *p_lo = is_r ? P[q] : P[(q + 1) % 3];
            const double *p_hi = is_r ? P[(q + 1) % 3] : P[q];
            const double mx = (p_lo[0] + p_hi[0]) / 2.0, mz = (p_lo[1] + p_hi[1]) / 2.0;
            if (is_r)
                m.hR[i] = (ux - mx) * nx + (uz - mz) * nz;
            else
                m.hL[i] = (mx - ux) * nx + (mz - uz) * nz;
        }
    }

    // 5. dual lengths and the Delaunay requirement d_i > dual_tol |e_i| on interior edges
    m.d.resize(ne);
    for (int64_t i = 0; i < ne; ++i) {
        m.d[i] = m.hR[i] + m.hL[i];
        if (m.interior(i) && !(m.d[i] > dom.dual_tol * m.elen[i]))
            return fail(TYEE_ENOTDELAUNAY, "edge " + std::to_string(i) + " (nodes " +
                                               std::to_string(m.edge[2 * i]) + "-" +
                                               std::to_string(m.edge[2 * i + 1]) +
                                               ") has a non-positive dual length");
    }
    m.perm_t.resize(nt);
    m.perm_e.resize(ne);
    std::iota(m.perm_t.begin(), m.perm_t.end(), 0);
    std::iota(m.perm_e.begin(), m.perm_e.end(), 0);
    return TYEE_OK;
}

// ---------------------------------------------------------------------------------------
// locality numbering
// ---------------------------------------------------------------------------------------

namespace {

void sort_by_key(std::vector<std::pair<uint64_t, int32_t>> &keyed, std::vector<int32_t> &perm) {
    std::sort(keyed.begin(), keyed.end());
    perm.resize(keyed.size());
    for (size_t r = 0; r < keyed.size(); ++r) perm[r] = keyed[r].second;
}

void number_edges_by_first_use(const Mesh &m, std::vector<int32_t> &perm_e) {
    std::vector<uint8_t> taken(m.ne, 0);
    perm_e.clear();
    perm_e.reserve(m.ne);
    for (int64_t r = 0; r < m.nt; ++r)
        for (int q = 0; q < 3; ++q) {
            int32_t i = m.A[3 * m.perm_t[r] + q];
            if (!taken[i]) {
                taken[i] = 1;
                perm_e.push_back(i);
            }
        }
}

uint32_t quantise(double c, double period) {
    double q = std::floor(c / period * 65536.0);
    return uint32_t(std::min(65535.0, std::max(0.0, q)));
}

struct DualGraph {
    const Mesh &m;
    int deg(int32_t j) const {
        return m.interior(m.A[3 * j]) + m.interior(m.A[3 * j + 1]) + m.interior(m.A[3 * j + 2]);
    }
    int32_t across(int32_t j, int q) const {
        int32_t i = m.A[3 * j + q];
        if (!m.interior(i)) return -1;
        return m.R[i] == j ? m.L[i] : m.R[i];
    }
    bool before(int32_t a, int32_t b) const {  // (degree, id) order
        int da = deg(a), db = deg(b);
        return da != db ? da < db : a < b;
    }
};

// Breadth-first sweep from root; returns its eccentricity and the (degree, id)-smallest
// triangle of the last level. `depth` must be all -1 on entry and is restored.
int64_t sweep(const DualGraph &g, int32_t root, std::vector<int64_t> &depth,
              std::vector<int32_t> &fifo, int32_t *deepest) {
    size_t head = 0;
    fifo.clear();
    fifo.push_back(root);
    depth[root] = 0;
    while (head < fifo.size()) {
        int32_t j = fifo[head++];
        for (int q = 0; q < 3; ++q) {
            int32_t k = g.across(j, q);
            if (k >= 0 && depth[k] < 0) {
                depth[k] = depth[j] + 1;
                fifo.push_back(k);
            }
        }
    }
    int64_t ecc = depth[fifo.back()];
    int32_t best = -1;
    for (int32_t j : fifo)
        if (depth[j] == ecc && (best < 0 || g.before(j, best))) best = j;
    for (int32_t j : fifo) depth[j] = -1;
    *deepest = best;
    return ecc;
}

void reverse_cuthill_mckee(const Mesh &m, std::vector<int32_t> &perm_t) {
    DualGraph g{m};
    const int64_t nt = m.nt;
    std::vector<int64_t> depth(nt, -1);
    std::vector<int32_t> fifo;
    std::vector<uint8_t> placed(nt, 0);
    std::vector<int32_t> cm;
    cm.reserve(nt);
    int32_t scan_deg_min = 0;
    while (int64_t(cm.size()) < nt) {
        // lowest (degree, id) triangle not yet placed
        int32_t root = -1;
        for (int32_t j = 0; j < nt; ++j)
            if (!placed[j] && (root < 0 || g.deg(j) < g.deg(root))) {
                root = j;
                if (g.deg(j) == scan_deg_min) break;
            }
        // George-Liu: move to the far end while the eccentricity grows
        int32_t cand;
        int64_t ecc = sweep(g, root, depth, fifo, &cand);
        while (true) {
            int32_t next;
            int64_t e2 = sweep(g, cand, depth, fifo, &next);
            if (e2 <= ecc) break;
            root = cand;
            ecc = e2;
            cand = next;
        }
        size_t head = cm.size();
        cm.push_back(root);
        placed[root] = 1;
        while (head < cm.size()) {
            int32_t j = cm[head++];
            int32_t nb[3];
            int cnt = 0;
            for (int q = 0; q < 3; ++q) {
                int32_t k = g.across(j, q);
                if (k >= 0 && !placed[k] && std::find(nb, nb + cnt, k) == nb + cnt) nb[cnt++] = k;
            }
            std::sort(nb, nb + cnt, [&](int32_t a, int32_t b) { return g.before(a, b); });
            for (int c = 0; c < cnt; ++c) {
                placed[nb[c]] = 1;
                cm.push_back(nb[c]);
            }
        }
    }
    perm_t.assign(cm.rbegin(), cm.rend());
}

}  // namespace

int reorder_mesh(Mesh &m, int32_t kind, uint64_t seed) {
    const int64_t nt = m.nt, ne = m.ne;
    switch (kind) {
    case TYEE_ORDER_NONE:
        m.perm_t.resize(nt);
        m.perm_e.resize(ne);
        std::iota(m.perm_t.begin(), m.perm_t.end(), 0);
        std::iota(m.perm_e.begin(), m.perm_e.end(), 0);
        break;
    case TYEE_ORDER_RANDOM: {
        std::vector<std::pair<uint64_t, int32_t>> keyed(nt);
        for (int64_t j = 0; j < nt; ++j) keyed[j] = {splitmix64(seed + uint64_t(j)), int32_t(j)};
        sort_by_key(keyed, m.perm_t);
        keyed.resize(ne);
        for (int64_t i = 0; i < ne; ++i) keyed[i] = {splitmix64(seed + uint64_t(nt) + uint64_t(i)), int32_t(i)};
        sort_by_key(keyed, m.perm_e);
        break;
    }
    case TYEE_ORDER_MORTON: {
        std::vector<std::pair<uint64_t, int32_t>> keyed(nt);
        for (int64_t j = 0; j < nt; ++j) {
            const int32_t *v = &m.tri[3 * j];
            double c[2];
            for (int ax = 0; ax < 2; ++ax) {
                const double period = ax ? m.Ly : m.Lx;
                const double xa = m.xy[2 * v[0] + ax], xb = m.xy[2 * v[1] + ax], xc = m.xy[2 * v[2] + ax];
                if (m.periodic) {
                    double ub = min_image(xb - xa, period, true), uc = min_image(xc - xa, period, true);
                    double p = xa + (ub + uc) / 3.0;
                    c[ax] = p - period * std::floor(p / period);
                } else {
                    c[ax] = ((xa + xb) + xc) / 3.0;
                }
            }
            keyed[j] = {morton_key(quantise(c[0], m.Lx), quantise(c[1], m.Ly)), int32_t(j)};
        }
        sort_by_key(keyed, m.perm_t);
        number_edges_by_first_use(m, m.perm_e);
        break;
    }
    case TYEE_ORDER_RCM:
        reverse_cuthill_mckee(m, m.perm_t);
        number_edges_by_first_use(m, m.perm_e);
        break;
    default:
        return fail(TYEE_EINVAL, "unknown ordering");
    }
    m.order_kind = kind;
    return TYEE_OK;
}

void dual_vectors(const Mesh &m, std::vector<double> &out) {
    out.assign(2 * m.ne, 0.0);
    for (int64_t i = 0; i < m.ne; ++i) {
        if (!m.interior(i)) continue;
        out[2 * i] = min_image(m.O[2 * m.R[i]] - m.O[2 * m.L[i]], m.Lx, m.periodic);
        out[2 * i + 1] = min_image(m.O[2 * m.R[i] + 1] - m.O[2 * m.L[i] + 1], m.Ly, m.periodic);
    }
}

void edge_features(const Mesh &m, std::vector<double> &out) {
    const int64_t nt = m.nt, ne = m.ne;
    // per triangle: the angle opposite each local side, and circumradius / shortest side
    std::vector<double> opp(3 * nt), rho(nt);
    double mean_area = 0.0;
    for (int64_t j = 0; j < nt; ++j) mean_area += m.S[j];
    mean_area /= double(nt);
    for (int64_t j = 0; j < nt; ++j) {
        const int32_t *v = &m.tri[3 * j];
        double P[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        for (int q = 1; q < 3; ++q) {
            P[q][0] = min_image(m.xy[2 * v[q]] - m.xy[2 * v[0]], m.Lx, m.periodic);
            P[q][1] = min_image(m.xy[2 * v[q] + 1] - m.xy[2 * v[0] + 1], m.Ly, m.periodic);
        }
        double shortest = INFINITY;
        for (int q = 0; q < 3; ++q) {
            const double *a = P[q], *b = P[(q + 1) % 3], *w = P[(q + 2) % 3];
            shortest = std::min(shortest, std::hypot(b[0] - a[0], b[1] - a[1]));
            const double ux = a[0] - w[0], uz = a[1] - w[1], vx = b[0] - w[0], vz = b[1] - w[1];
            opp[3 * j + q] = std::atan2(std::fabs(ux * vz - uz * vx), ux * vx + uz * vz);
        }
        const double ox = min_image(m.O[2 * j] - m.xy[2 * v[0]], m.Lx, m.periodic);
        const double oz = min_image(m.O[2 * j + 1] - m.xy[2 * v[0] + 1], m.Ly, m.periodic);
        rho[j] = std::hypot(ox, oz) / shortest;
    }
    std::vector<double> angR(ne, 0.0), angL(ne, 0.0);
    for (int64_t k = 0; k < 3 * nt; ++k) (m.sgn[k] > 0 ? angR : angL)[m.A[k]] = opp[k];
    out.assign(size_t(kFeatures) * ne, 0.0);
    for (int64_t i = 0; i < ne; ++i) {
        const int32_t r = m.R[i] >= 0 ? m.R[i] : m.L[i], l = m.L[i] >= 0 ? m.L[i] : m.R[i];
        const double ar = m.R[i] >= 0 ? angR[i] : angL[i], al = m.L[i] >= 0 ? angL[i] : angR[i];
        double *f = &out[size_t(kFeatures) * i];
        f[0] = m.d[i] / m.elen[i];
        f[1] = std::min(ar, al);
        f[2] = std::max(ar, al);
        f[3] = std::min(rho[r], rho[l]);
        f[4] = std::max(rho[r], rho[l]);
        f[5] = std::fabs(m.hR[i] - m.hL[i]) / m.d[i];
        f[6] = m.elen[i] / std::sqrt(mean_area);
        f[7] = std::fabs(m.S[r] - m.S[l]) / (m.S[r] + m.S[l]);
    }
}

void rq_phase_errors(const Mesh &m, const double *gamma, double dt, const double *waves, int64_t n_waves,
                     double *out) {
    double area = 0.0;
    for (int64_t j = 0; j < m.nt; ++j) area += m.S[j];
    std::vector<double> dv;
    dual_vectors(m, dv);
    const int64_t chunks = 256;
    std::vector<double> part(size_t(chunks) * n_waves, 0.0);
    parallel_for(chunks, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            double *acc = &part[size_t(c) * n_waves];
            for (int64_t i = m.ne * c / chunks; i < m.ne * (c + 1) / chunks; ++i) {
                if (!m.interior(i)) continue;
                const double g = gamma ? gamma[i] : 1.0;
                const double base = g * g * (m.elen[i] / m.d[i]) * 4.0;
                for (int64_t w = 0; w < n_waves; ++w) {
                    const double s = std::sin(0.5 * (waves[2 * w] * dv[2 * i] + waves[2 * w + 1] * dv[2 * i + 1]));
                    acc[w] += base * s * s;
                }
            }
        }
    }, m.ne * n_waves);
    for (int64_t w = 0; w < n_waves; ++w) {
        double sum = 0.0;
        for (int64_t c = 0; c < chunks; ++c) sum += part[size_t(c) * n_waves + w];
        const double om = std::sqrt(sum / area);
        out[w] = 2.0 / dt * std::asin(om * dt / 2.0) / std::hypot(waves[2 * w], waves[2 * w + 1]) - 1.0;
    }
}

int merge_meshes(const std::vector<const Mesh *> &parts, Mesh &out) {
    if (parts.empty()) return fail(TYEE_EINVAL, "no meshes to merge");
    out = Mesh();
    int64_t nv = 0, ne = 0, nt = 0;
    for (const Mesh *p : parts) {
        nv += p->nv;
        ne += p->ne;
        nt += p->nt;
    }
    if (nv > INT32_MAX || 3 * nt > INT32_MAX) return fail(TYEE_EINVAL, "batch too large for int32 ids");
    out.periodic = parts[0]->periodic;
    out.Lx = parts[0]->Lx;
    out.Ly = parts[0]->Ly;
    out.order_kind = parts[0]->order_kind;
    int32_t ov = 0, oe = 0, ot = 0;
    auto shift = [](int32_t v, int32_t off) { return v >= 0 ? v + off : v; };
    for (const Mesh *p : parts) {
        out.xy.insert(out.xy.end(), p->xy.begin(), p->xy.end());
        for (int32_t v : p->tri) out.tri.push_back(v + ov);
        for (int32_t v : p->edge) out.edge.push_back(v + ov);
        for (int32_t v : p->R) out.R.push_back(shift(v, ot));
        for (int32_t v : p->L) out.L.push_back(shift(v, ot));
        for (int32_t v : p->A) out.A.push_back(v + oe);
        out.sgn.insert(out.sgn.end(), p->sgn.begin(), p->sgn.end());
        out.evec.insert(out.evec.end(), p->evec.begin(), p->evec.end());
        out.elen.insert(out.elen.end(), p->elen.begin(), p->elen.end());
        out.hR.insert(out.hR.end(), p->hR.begin(), p->hR.end());
        out.hL.insert(out.hL.end(), p->hL.begin(), p->hL.end());
        out.d.insert(out.d.end(), p->d.begin(), p->d.end());
        out.S.insert(out.S.end(), p->S.begin(), p->S.end());
        out.O.insert(out.O.end(), p->O.begin(), p->O.end());
        out.C.insert(out.C.end(), p->C.begin(), p->C.end());
        out.node_outer.insert(out.node_outer.end(), p->node_outer.begin(), p->node_outer.end());
        for (int32_t v : p->perm_t) out.perm_t.push_back(v + ot);
        for (int32_t v : p->perm_e) out.perm_e.push_back(v + oe);
        out.nb += p->nb;
        ov += int32_t(p->nv);
        oe += int32_t(p->ne);
        ot += int32_t(p->nt);
    }
    out.nv = nv;
    out.ne = ne;
    out.nt = nt;
    return TYEE_OK;
}

// ---------------------------------------------------------------------------------------
// omega_max^2 by normalised iteration on K = -L_E L_B in the S-weighted product
// ---------------------------------------------------------------------------------------

int power_iteration(const Mesh &m, const double *gamma, int64_t max_iter, double rtol,
                    uint64_t seed, double *lambda, int64_t *iters) {
    const int64_t nt = m.nt, ne = m.ne;
    if (max_iter < 2 || !(rtol >= 0.0)) return fail(TYEE_EINVAL, "max_iter >= 2 and rtol >= 0 required");
    // K x = (1/S_j) sum over interior edges of j of w_i (x_j - x_other), w = gamma^2 |e|/d
    std::vector<double> w(ne, 0.0);
    for (int64_t i = 0; i < ne; ++i)
        if (m.interior(i)) {
            double g = gamma ? gamma[i] : 1.0;
            w[i] = g * g * m.elen[i] / m.d[i];
        }
    std::vector<double> x(nt), y(nt);
    for (int64_t j = 0; j < nt; ++j) {
        double u = double(splitmix64(seed + uint64_t(j)) >> 11) * 0x1.0p-53;
        x[j] = 2.0 * u - 1.0;
    }
    const int64_t chunks = 256;
    std::vector<double> part(3 * chunks);
    double lam = 0.0, prev = 0.0;
    for (int64_t it = 1; it <= max_iter; ++it) {
        parallel_for(chunks, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c) {
                double sxy = 0.0, sxx = 0.0, syy = 0.0;
                for (int64_t j = nt * c / chunks; j < nt * (c + 1) / chunks; ++j) {
                    double acc = 0.0;
                    for (int q = 0; q < 3; ++q) {
                        int32_t i = m.A[3 * j + q];
                        if (w[i] == 0.0) continue;
                        int32_t o = m.R[i] == j ? m.L[i] : m.R[i];
                        acc += w[i] * (x[j] - x[o]);
                    }
                    double yj = acc / m.S[j];
                    y[j] = yj;
                    sxy += m.S[j] * x[j] * yj;
                    sxx += m.S[j] * x[j] * x[j];
                    syy += m.S[j] * yj * yj;
                }
                part[3 * c] = sxy;
                part[3 * c + 1] = sxx;
                part[3 * c + 2] = syy;
            }
        }, nt);
        double sxy = 0.0, sxx = 0.0, syy = 0.0;
        for (int64_t c = 0; c < chunks; ++c) {
            sxy += part[3 * c];
            sxx += part[3 * c + 1];
            syy += part[3 * c + 2];
        }
        lam = sxy / sxx;
        const double inv = 1.0 / std::sqrt(syy);
        parallel_for(nt, [&](int64_t a, int64_t b) {
            for (int64_t j = a; j < b; ++j) x[j] = y[j] * inv;
        });
        if (it > 1 && std::fabs(lam - prev) <= rtol * lam) {
            *lambda = lam;
            if (iters) *iters = it;
            return TYEE_OK;
        }
        prev = lam;
    }
    *lambda = lam;
    if (iters) *iters = max_iter;
    return fail(TYEE_ENOTCONVERGED, "power iteration did not converge");
}

namespace {
double flip_mi(double d, double L, bool periodic) { return periodic ? d - L * std::nearbyint(d / L) : d; }
}  // namespace

// Lawson flips until every interior edge passes the empty-circle test (with a relative
// tolerance, so that cocircular quads are left alone).  Triangles stay counter-clockwise.
int lawson_flip(const std::vector<double> &xy, std::vector<int32_t> &tri, bool periodic, double Lx, double Ly,
                int64_t nv, int64_t max_flips, int64_t *n_flips) {
    const int64_t nt = int64_t(tri.size()) / 3;
    auto key = [nv](int64_t a, int64_t b) { return a < b ? a * nv + b : b * nv + a; };
    std::unordered_map<int64_t, std::pair<int64_t, int64_t>> sides;  // edge -> (3 t + q, 3 t' + q')
    sides.reserve(size_t(3 * nt));
    for (int64_t j = 0; j < nt; ++j)
        for (int q = 0; q < 3; ++q) {
            const int64_t k = key(tri[3 * j + q], tri[3 * j + (q + 1) % 3]);
            auto it = sides.find(k);
            if (it == sides.end()) sides.emplace(k, std::make_pair(3 * j + q, int64_t(-1)));
            else it->second.second = 3 * j + q;
        }
    std::vector<int64_t> stack;
    stack.reserve(sides.size());
    for (auto &kv : sides)
        if (kv.second.second >= 0) stack.push_back(kv.first);
    std::sort(stack.begin(), stack.end());  // a fixed order, whatever the hash map's
    auto rel = [&](int32_t from, int32_t to, double &dx, double &dy) {
        dx = flip_mi(xy[2 * to] - xy[2 * from], Lx, periodic);
        dy = flip_mi(xy[2 * to + 1] - xy[2 * from + 1], Ly, periodic);
    };
    auto replace = [&](int64_t k, int64_t old_s, int64_t new_s) {
        auto &pr = sides[k];
        if (pr.first == old_s) pr.first = new_s;
        else if (pr.second == old_s) pr.second = new_s;
    };
    int64_t flips = 0;
    while (!stack.empty() && flips < max_flips) {
        const int64_t k = stack.back();
        stack.pop_back();
        auto it = sides.find(k);
        if (it == sides.end() || it->second.second < 0) continue;
        const int64_t s1 = it->second.first, s2 = it->second.second;
        const int64_t t1 = s1 / 3, q1 = s1 % 3, t2 = s2 / 3, q2 = s2 % 3;
        const int32_t u = tri[3 * t1 + q1], v = tri[3 * t1 + (q1 + 1) % 3], o1 = tri[3 * t1 + (q1 + 2) % 3];
        const int32_t o2 = tri[3 * t2 + (q2 + 2) % 3];
        if (o1 == o2 || sides.count(key(o1, o2))) continue;  // the new diagonal exists already
        // in-circle test of o2 against the circle through u, v, o1 (counter-clockwise)
        double bx, by, cx, cy, dx, dy;
        rel(u, v, bx, by);
        rel(u, o1, cx, cy);
        rel(u, o2, dx, dy);
        // with u at the origin: incircle = -| b |b|^2 ; c |c|^2 ; d |d|^2 | (rows x, y, x^2 + y^2),
        // positive when o2 is inside the circle
        const double b2 = bx * bx + by * by, c2 = cx * cx + cy * cy, d2 = dx * dx + dy * dy;
        const double incircle =
            -(bx * (cy * d2 - c2 * dy) - by * (cx * d2 - c2 * dx) + b2 * (cx * dy - cy * dx));
        const double scale = std::max(b2, std::max(c2, d2));
        if (!(incircle > 1e-12 * scale * scale)) continue;
        // flip u-v to o1-o2: t1 = (o1, u, o2), t2 = (o2, v, o1)
        const int64_t k_uo2 = key(u, o2), k_vo1 = key(v, o1), k_o1u = key(o1, u), k_o2v = key(o2, v);
        // sides before: t1: (u,v) q1, (v,o1) q1+1, (o1,u) q1+2; t2: (v,u) q2, (u,o2) q2+1, (o2,v) q2+2
        const int64_t s_vo1 = 3 * t1 + (q1 + 1) % 3, s_o1u = 3 * t1 + (q1 + 2) % 3;
        const int64_t s_uo2 = 3 * t2 + (q2 + 1) % 3, s_o2v = 3 * t2 + (q2 + 2) % 3;
        tri[3 * t1] = o1;
        tri[3 * t1 + 1] = u;
        tri[3 * t1 + 2] = o2;
        tri[3 * t2] = o2;
        tri[3 * t2 + 1] = v;
        tri[3 * t2 + 2] = o1;
        // sides after: t1: (o1,u) 0, (u,o2) 1, (o2,o1) 2; t2: (o2,v) 0, (v,o1) 1, (o1,o2) 2
        replace(k_o1u, s_o1u, 3 * t1 + 0);
        replace(k_uo2, s_uo2, 3 * t1 + 1);
        replace(k_o2v, s_o2v, 3 * t2 + 0);
        replace(k_vo1, s_vo1, 3 * t2 + 1);
        sides.erase(it);
        sides.emplace(key(o1, o2), std::make_pair(3 * t1 + 2, 3 * t2 + 2));
        for (int64_t kk : {k_uo2, k_vo1, k_o1u, k_o2v}) stack.push_back(kk);
        ++flips;
    }
    *n_flips = flips;
    if (!stack.empty()) return fail(TYEE_EUNSTABLE, "Lawson flips did not finish within the flip limit");
    return TYEE_OK;
}


}  // namespace tyee

// ---------------------------------------------------------------------------------------
// C ABI: mesh
// ---------------------------------------------------------------------------------------

extern "C" {

const char *tyee_last_error(void) { return tyee::g_last_error.c_str(); }

int tyee_mesh_create(const double *xy, int64_t n_nodes, const int32_t *tri, int64_t n_tris,
                     const tyee_domain *dom, tyee_mesh **out) {
    if (!out || !dom) return tyee::fail(TYEE_EINVAL, "null argument");
    *out = nullptr;
    try {
        auto *h = new tyee_mesh();
        int rc = tyee::build_mesh(xy, n_nodes, tri, n_tris, *dom, h->m);
        if (rc != TYEE_OK) {
            delete h;
            return rc;
        }
        *out = h;
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return tyee::fail(TYEE_ENOMEM, "host allocation failed");
    }
}

int tyee_mesh_reorder(tyee_mesh *mesh, int32_t kind, uint64_t seed) {
    if (!mesh) return tyee::fail(TYEE_EINVAL, "null mesh");
    try {
        return tyee::reorder_mesh(mesh->m, kind, seed);
    } catch (const std::bad_alloc &) {
        return tyee::fail(TYEE_ENOMEM, "host allocation failed");
    }
}

int tyee_mesh_query(const tyee_mesh *mesh, tyee_mesh_info *out) {
    if (!mesh || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    const tyee::Mesh &m = mesh->m;
    tyee_mesh_info info{};
    info.n_nodes = m.nv;
    info.n_edges = m.ne;
    info.n_tris = m.nt;
    info.n_boundary_edges = m.nb;
    info.min_dual_ratio = INFINITY;
    info.max_dual_ratio = 0.0;
    for (int64_t i = 0; i < m.ne; ++i) {
        info.sum_dual_area += m.elen[i] * m.d[i] / 2.0;
        if (!m.interior(i)) continue;
        double r = m.d[i] / m.elen[i];
        info.min_dual_ratio = std::min(info.min_dual_ratio, r);
        info.max_dual_ratio = std::max(info.max_dual_ratio, r);
    }
    for (int64_t j = 0; j < m.nt; ++j) {
        info.sum_area += m.S[j];
        // circumcentre outside the triangle <=> some half dual length is negative
        bool out_side = false;
        for (int q = 0; q < 3; ++q) {
            int32_t i = m.A[3 * j + q];
            double h = m.sgn[3 * j + q] > 0 ? m.hR[i] : m.hL[i];
            out_side |= h < 0.0;
        }
        info.n_obtuse += out_side;
    }
    *out = info;
    return TYEE_OK;
}

int tyee_mesh_view(const tyee_mesh *mesh, tyee_mesh_arrays *out) {
    if (!mesh || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    const tyee::Mesh &m = mesh->m;
    out->tri = m.tri.data();
    out->edge_nodes = m.edge.data();
    out->R = m.R.data();
    out->L = m.L.data();
    out->A = m.A.data();
    out->sgn = m.sgn.data();
    out->elen = m.elen.data();
    out->evec = m.evec.data();
    out->hR = m.hR.data();
    out->hL = m.hL.data();
    out->d = m.d.data();
    out->S = m.S.data();
    out->O = m.O.data();
    out->C = m.C.data();
    out->perm_t = m.perm_t.data();
    out->perm_e = m.perm_e.data();
    return TYEE_OK;
}

int tyee_mesh_cfl(const tyee_mesh *mesh, const double *gamma, int64_t max_iter, double rtol,
                  uint64_t seed, double *lambda, int64_t *iters) {
    if (!mesh || !lambda) return tyee::fail(TYEE_EINVAL, "null argument");
    try {
        return tyee::power_iteration(mesh->m, gamma, max_iter, rtol, seed, lambda, iters);
    } catch (const std::bad_alloc &) {
        return tyee::fail(TYEE_ENOMEM, "host allocation failed");
    }
}

int tyee_mesh_features(const tyee_mesh *mesh, double *out) {
    if (!mesh || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    std::vector<double> f;
    tyee::edge_features(mesh->m, f);
    std::copy(f.begin(), f.end(), out);
    return TYEE_OK;
}

int tyee_mesh_phase_error_rq(const tyee_mesh *mesh, const double *gamma, double dt, const double *waves,
                             int64_t n_waves, double *out) {
    if (!mesh || !waves || !out || n_waves <= 0 || !(dt > 0.0)) return tyee::fail(TYEE_EINVAL, "bad arguments");
    for (int64_t w = 0; w < n_waves; ++w)
        if (waves[2 * w] == 0.0 && waves[2 * w + 1] == 0.0) return tyee::fail(TYEE_EINVAL, "zero wavevector");
    tyee::rq_phase_errors(mesh->m, gamma, dt, waves, n_waves, out);
    return TYEE_OK;
}

void tyee_mesh_destroy(tyee_mesh *mesh) { delete mesh; }

}  // extern "C"

extern "C" int tyee_mesh_flip(const double *xy, int64_t n_nodes, int32_t *tri, int64_t n_tris,
                              const tyee_domain *dom, int64_t *flips) {
    using namespace tyee;
    if (!xy || !tri || !dom || n_nodes <= 0 || n_tris <= 0) return fail(TYEE_EINVAL, "null or empty argument");
    if (n_nodes > INT32_MAX || 3 * n_tris > INT32_MAX) return fail(TYEE_EINVAL, "mesh too large for int32 ids");
    const bool periodic = dom->kind == TYEE_PERIODIC;
    std::vector<double> p(xy, xy + 2 * n_nodes);
    std::vector<int32_t> t(tri, tri + 3 * n_tris);
    for (int64_t j = 0; j < n_tris; ++j) {
        for (int q = 0; q < 3; ++q)
            if (t[3 * j + q] < 0 || t[3 * j + q] >= n_nodes) return fail(TYEE_EINVAL, "node id out of range");
        const int32_t a = t[3 * j], b = t[3 * j + 1], c = t[3 * j + 2];
        const double bx = flip_mi(p[2 * b] - p[2 * a], dom->Lx, periodic), by = flip_mi(p[2 * b + 1] - p[2 * a + 1], dom->Ly, periodic);
        const double cx = flip_mi(p[2 * c] - p[2 * a], dom->Lx, periodic), cy = flip_mi(p[2 * c + 1] - p[2 * a + 1], dom->Ly, periodic);
        const double o = bx * cy - by * cx;
        if (o == 0.0) return fail(TYEE_EDEGENERATE, "degenerate triangle");
        if (o < 0.0) std::swap(t[3 * j + 1], t[3 * j + 2]);  // counter-clockwise
    }
    int64_t n = 0;
    const int rc = lawson_flip(p, t, periodic, dom->Lx, dom->Ly, n_nodes, 50 * n_tris, &n);
    if (flips) *flips = n;
    if (rc) return rc;
    std::copy(t.begin(), t.end(), tri);
    return TYEE_OK;
}
