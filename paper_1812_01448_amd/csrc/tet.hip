// Device stepping of the three-dimensional scheme on tetrahedra (the paper's Conclusion: E on
// edges, B on faces).  The device holds line integrals, so that each update needs one
// coefficient per cell:
//   e_e = |e| E_e           (E along the edge),
//   h_f = d_f B_f           (B along the dual edge that crosses face f; B_f itself on a wall
//                            face, which never changes);
// Faraday on an inner face:  h_f -= (dt d_f / A_f) (e_ab + e_bc - e_ac),
// Ampere on an inner edge:   e_e += (dt |e| / A*_e) sum over the faces around it of s h_f,
// leap-frog, E then B, as in two dimensions.  Wall edges (the conducting box) keep e = 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "sim.hpp"
#include "tet.hpp"

namespace tyee {
namespace {

// Faraday: every face, wall faces with g = 0.  A face's circuit a -> b -> c runs along (a, b)
// and (b, c) and against (a, c), the fixed order of its three edge ids.
template <typename T>
__global__ void k_tet_face(int32_t nf, const int32_t *__restrict__ eab, const int32_t *__restrict__ ebc,
                           const int32_t *__restrict__ eac, const T *__restrict__ g, const T *__restrict__ e,
                           T *__restrict__ h) {
    const int f = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    h[f] = h[f] - g[f] * (e[eab[f]] + e[ebc[f]] - e[eac[f]]);
}

// Ampere.  The faces around the edges are held in slices of kSlice = 64 edges (one wavefront):
// slice s has width w_s (its longest row) and its entries slot-major at so_s + k kSlice + lane,
// so every load of a wave is one contiguous run; each entry is f or ~f (a circuit against the
// edge), padding and wall edges read the zero kept at h[nf].
constexpr int kSlice = 64;

template <typename T, int W>
__device__ __forceinline__ T slice_row(const int32_t *__restrict__ r, const T *__restrict__ h, int lane) {
    int32_t id[W];
#pragma unroll
    for (int k = 0; k < W; ++k) id[k] = r[k * kSlice + lane];
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const T v = h[id[k] ^ (id[k] >> 31)];
        acc += id[k] < 0 ? -v : v;
    }
    return acc;
}

template <typename T>
__global__ void k_tet_edge(int32_t ne, const int32_t *__restrict__ sw, const int32_t *__restrict__ so,
                           const int32_t *__restrict__ ids, const T *__restrict__ a, const T *__restrict__ h,
                           T *__restrict__ e) {
    const int i = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int s = i / kSlice, lane = i % kSlice;      // kBlock is a multiple of kSlice: s is the wave's
    const int w = sw[s];
    if (w == 0) return;
    const int32_t *r = ids + so[s];
    T acc;
    switch (w) {
    case 1: acc = slice_row<T, 1>(r, h, lane); break;
    case 2: acc = slice_row<T, 2>(r, h, lane); break;
    case 3: acc = slice_row<T, 3>(r, h, lane); break;
    case 4: acc = slice_row<T, 4>(r, h, lane); break;
    case 5: acc = slice_row<T, 5>(r, h, lane); break;
    case 6: acc = slice_row<T, 6>(r, h, lane); break;
    case 7: acc = slice_row<T, 7>(r, h, lane); break;
    case 8: acc = slice_row<T, 8>(r, h, lane); break;
    default:
        acc = T(0);
        for (int k = 0; k < w; ++k) {
            const int32_t id = r[k * kSlice + lane];
            const T v = h[id ^ (id >> 31)];
            acc += id < 0 ? -v : v;
        }
    }
    e[i] = e[i] + a[i] * acc;
}
static_assert(tyee::kBlock % kSlice == 0, "a work-group holds whole slices");

}  // namespace
}  // namespace tyee

struct tyee_tet_sim {
    bool f64 = false;
    double dt = 0.0;
    int64_t ne = 0, nf = 0;
    std::vector<double> escale, hscale;   // |e| per edge; d_f per inner face, 1 per wall face
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tyee::DeviceBuffer e, h, g, a, eab, ebc, eac, sw, so, ids;
    int32_t graph_steps = 8;
    hipGraphExec_t graph = nullptr;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    double ms_edge = 0.0, ms_face = 0.0;
    int64_t timed = 0;
    ~tyee_tet_sim() {
        if (graph) (void)hipGraphExecDestroy(graph);
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace tyee {
namespace {

template <typename T>
int upload_tet(tyee_tet_sim &s, const TetMesh &m) {
    const size_t ts = sizeof(T);
    std::vector<T> g(m.nf), a(m.ne);
    std::vector<int32_t> eab(m.nf), ebc(m.nf), eac(m.nf);
    for (int64_t f = 0; f < m.nf; ++f) {
        eab[f] = m.face_edge[3 * f];
        ebc[f] = m.face_edge[3 * f + 1];
        eac[f] = m.face_edge[3 * f + 2];
        g[f] = m.inner_face[f] ? T(s.dt * m.d[f] / m.farea[f]) : T(0);
    }
    for (int64_t i = 0; i < m.ne; ++i) a[i] = m.inner_edge[i] ? T(s.dt * m.elen[i] / m.dual_area[i]) : T(0);
    // sliced rows: width and start of every slice of kSlice edges, entries slot-major, padding
    // pointing at the zero h[nf]
    const int64_t ns = (m.ne + kSlice - 1) / kSlice;
    std::vector<int32_t> sw(ns), so(ns);
    int64_t slots = 0;
    for (int64_t q = 0; q < ns; ++q) {
        int64_t w = 0;
        for (int64_t i = q * kSlice; i < std::min(m.ne, (q + 1) * kSlice); ++i)
            w = std::max(w, m.ef_off[i + 1] - m.ef_off[i]);
        sw[q] = int32_t(w);
        so[q] = int32_t(slots);
        slots += w * kSlice;
        if (slots >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "too many edge-face entries for one table");
    }
    std::vector<int32_t> ids(std::max<int64_t>(slots, 1), int32_t(m.nf));
    for (int64_t i = 0; i < m.ne; ++i) {
        const int64_t q = i / kSlice, lane = i % kSlice;
        for (int64_t k = 0; k < m.ef_off[i + 1] - m.ef_off[i]; ++k) ids[so[q] + k * kSlice + lane] = m.ef[m.ef_off[i] + k];
    }
    auto put = [&](DeviceBuffer &b, const void *src, size_t bytes) -> int {
        int r = b.alloc(std::max<size_t>(bytes, 16));
        if (r) return r;
        if (src) TYEE_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s.stream));
        else TYEE_HIP(hipMemsetAsync(b.p, 0, bytes, s.stream));
        return TYEE_OK;
    };
    int rc = 0;
    if ((rc = put(s.e, nullptr, m.ne * ts)) || (rc = put(s.h, nullptr, (m.nf + 1) * ts)) ||
        (rc = put(s.g, g.data(), m.nf * ts)) || (rc = put(s.a, a.data(), m.ne * ts)) ||
        (rc = put(s.eab, eab.data(), m.nf * 4)) || (rc = put(s.ebc, ebc.data(), m.nf * 4)) ||
        (rc = put(s.eac, eac.data(), m.nf * 4)) || (rc = put(s.sw, sw.data(), ns * 4)) ||
        (rc = put(s.so, so.data(), ns * 4)) || (rc = put(s.ids, ids.data(), ids.size() * 4)))
        return rc;
    TYEE_HIP(hipStreamSynchronize(s.stream));
    return TYEE_OK;
}

template <typename T>
void enqueue_edge(tyee_tet_sim &s) {
    const int32_t ne = int32_t(s.ne);
    hipLaunchKernelGGL(k_tet_edge<T>, dim3(unsigned(blocks_for(ne))), dim3(kBlock), 0, s.stream, ne,
                       s.sw.as<int32_t>(), s.so.as<int32_t>(), s.ids.as<int32_t>(), s.a.as<T>(), s.h.as<T>(),
                       s.e.as<T>());
}

template <typename T>
void enqueue_face(tyee_tet_sim &s) {
    const int32_t nf = int32_t(s.nf);
    hipLaunchKernelGGL(k_tet_face<T>, dim3(unsigned(blocks_for(nf))), dim3(kBlock), 0, s.stream, nf,
                       s.eab.as<int32_t>(), s.ebc.as<int32_t>(), s.eac.as<int32_t>(), s.g.as<T>(), s.e.as<T>(),
                       s.h.as<T>());
}

constexpr int64_t kTimedChunk = 256;

template <typename T>
int launch_timed(tyee_tet_sim &s, int64_t nsteps) {
    if (s.ev.empty()) {
        s.ev.assign(3 * kTimedChunk, nullptr);
        for (hipEvent_t &x : s.ev) TYEE_HIP(hipEventCreate(&x));
    }
    for (int64_t s0 = 0; s0 < nsteps; s0 += kTimedChunk) {
        const int64_t chunk = std::min(kTimedChunk, nsteps - s0);
        for (int64_t k = 0; k < chunk; ++k) {
            TYEE_HIP(hipEventRecord(s.ev[3 * k], s.stream));
            enqueue_edge<T>(s);
            TYEE_HIP(hipGetLastError());
            TYEE_HIP(hipEventRecord(s.ev[3 * k + 1], s.stream));
            enqueue_face<T>(s);
            TYEE_HIP(hipGetLastError());
            TYEE_HIP(hipEventRecord(s.ev[3 * k + 2], s.stream));
        }
        TYEE_HIP(hipEventSynchronize(s.ev[3 * (chunk - 1) + 2]));
        for (int64_t k = 0; k < chunk; ++k) {
            float x = 0.0f, y = 0.0f;
            TYEE_HIP(hipEventElapsedTime(&x, s.ev[3 * k], s.ev[3 * k + 1]));
            TYEE_HIP(hipEventElapsedTime(&y, s.ev[3 * k + 1], s.ev[3 * k + 2]));
            s.ms_edge += x;
            s.ms_face += y;
        }
        s.timed += chunk;
    }
    return TYEE_OK;
}

// Whole graphs of graph_steps steps (captured once: the buffers never move), the rest eager.
template <typename T>
int launch_tet(tyee_tet_sim &s, int64_t nsteps) {
    if (s.timing) return launch_timed<T>(s, nsteps);
    int64_t done = 0;
    if (s.graph_steps > 0 && nsteps >= s.graph_steps) {
        if (!s.graph) {
            TYEE_HIP(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
            for (int32_t k = 0; k < s.graph_steps; ++k) {
                enqueue_edge<T>(s);
                enqueue_face<T>(s);
            }
            hipGraph_t graph = nullptr;
            hipError_t err = hipStreamEndCapture(s.stream, &graph);
            if (err != hipSuccess) return fail(TYEE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(err));
            err = hipGraphInstantiate(&s.graph, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (err != hipSuccess) {
                s.graph = nullptr;
                return fail(TYEE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(err));
            }
        }
        for (; nsteps - done >= s.graph_steps; done += s.graph_steps) TYEE_HIP(hipGraphLaunch(s.graph, s.stream));
    }
    for (; done < nsteps; ++done) {
        enqueue_edge<T>(s);
        enqueue_face<T>(s);
    }
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

int tet_field(tyee_tet_sim *s, int32_t field, int64_t *n, DeviceBuffer **buf, const std::vector<double> **scale) {
    switch (field) {
    case TYEE_TET_E: *n = s->ne; *buf = &s->e; *scale = &s->escale; return TYEE_OK;
    case TYEE_TET_B: *n = s->nf; *buf = &s->h; *scale = &s->hscale; return TYEE_OK;
    default: return fail(TYEE_EINVAL, "field must be TYEE_TET_E or TYEE_TET_B");
    }
}

}  // namespace
}  // namespace tyee

extern "C" int tyee_tet_sim_create(const tyee_tet *mesh, int32_t prec, double dt, void *stream, tyee_tet_sim **out) {
    using namespace tyee;
    if (!mesh || !out) return fail(TYEE_EINVAL, "null argument");
    *out = nullptr;
    if (prec != TYEE_F32 && prec != TYEE_F64) return fail(TYEE_EINVAL, "prec must be TYEE_F32 or TYEE_F64");
    if (!(dt > 0.0)) return fail(TYEE_EINVAL, "dt must be positive");
    const TetMesh &m = mesh->m;
    try {
        std::unique_ptr<tyee_tet_sim> s(new tyee_tet_sim());
        s->f64 = prec == TYEE_F64;
        s->dt = dt;
        s->ne = m.ne;
        s->nf = m.nf;
        s->escale = m.elen;
        s->hscale.resize(m.nf);
        for (int64_t f = 0; f < m.nf; ++f) s->hscale[f] = m.inner_face[f] ? m.d[f] : 1.0;
        if (stream) {
            s->stream = static_cast<hipStream_t>(stream);
        } else {
            TYEE_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
            s->own_stream = true;
        }
        const int rc = s->f64 ? upload_tet<double>(*s, m) : upload_tet<float>(*s, m);
        if (rc) return rc;
        *out = s.release();
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

extern "C" int tyee_tet_sim_set_state(tyee_tet_sim *s, int32_t field, const double *values) {
    using namespace tyee;
    if (!s || !values) return fail(TYEE_EINVAL, "null argument");
    int64_t n = 0;
    DeviceBuffer *b = nullptr;
    const std::vector<double> *scale = nullptr;
    int rc = tet_field(s, field, &n, &b, &scale);
    if (rc) return rc;
    TYEE_HIP(hipStreamSynchronize(s->stream));
    if (s->f64) {
        std::vector<double> tmp(n);
        for (int64_t i = 0; i < n; ++i) tmp[i] = values[i] * (*scale)[i];
        TYEE_HIP(hipMemcpy(b->p, tmp.data(), size_t(n) * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> tmp(n);
        for (int64_t i = 0; i < n; ++i) tmp[i] = float(values[i] * (*scale)[i]);
        TYEE_HIP(hipMemcpy(b->p, tmp.data(), size_t(n) * 4, hipMemcpyHostToDevice));
    }
    return TYEE_OK;
}

extern "C" int tyee_tet_sim_get_state(tyee_tet_sim *s, int32_t field, double *values) {
    using namespace tyee;
    if (!s || !values) return fail(TYEE_EINVAL, "null argument");
    int64_t n = 0;
    DeviceBuffer *b = nullptr;
    const std::vector<double> *scale = nullptr;
    int rc = tet_field(s, field, &n, &b, &scale);
    if (rc) return rc;
    TYEE_HIP(hipStreamSynchronize(s->stream));
    if (s->f64) {
        TYEE_HIP(hipMemcpy(values, b->p, size_t(n) * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(n);
        TYEE_HIP(hipMemcpy(tmp.data(), b->p, size_t(n) * 4, hipMemcpyDeviceToHost));
        std::copy(tmp.begin(), tmp.end(), values);
    }
    for (int64_t i = 0; i < n; ++i) values[i] /= (*scale)[i];
    return TYEE_OK;
}

extern "C" int tyee_tet_sim_step(tyee_tet_sim *s, int64_t nsteps) {
    using namespace tyee;
    if (!s || nsteps < 0) return fail(TYEE_EINVAL, "null handle or negative step count");
    return s->f64 ? launch_tet<double>(*s, nsteps) : launch_tet<float>(*s, nsteps);
}

extern "C" int tyee_tet_sim_set_graph(tyee_tet_sim *s, int32_t steps) {
    if (!s) return tyee::fail(TYEE_EINVAL, "null argument");
    if (steps < 0 || steps > 1024) return tyee::fail(TYEE_EINVAL, "steps per graph must be in 0 .. 1024");
    if (s->graph) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) return tyee::fail(TYEE_EDEVICE, "hipStreamSynchronize failed");
        (void)hipGraphExecDestroy(s->graph);
        s->graph = nullptr;
    }
    s->graph_steps = steps;
    return TYEE_OK;
}

extern "C" int tyee_tet_sim_sync(tyee_tet_sim *s) {
    if (!s) return tyee::fail(TYEE_EINVAL, "null argument");
    if (hipStreamSynchronize(s->stream) != hipSuccess) return tyee::fail(TYEE_EDEVICE, "hipStreamSynchronize failed");
    return TYEE_OK;
}

extern "C" int tyee_tet_sim_set_timing(tyee_tet_sim *s, int32_t on) {
    if (!s) return tyee::fail(TYEE_EINVAL, "null argument");
    s->timing = on != 0;
    s->ms_edge = s->ms_face = 0.0;
    s->timed = 0;
    return TYEE_OK;
}

extern "C" int tyee_tet_sim_kernel_ms(const tyee_tet_sim *s, double out[2], int64_t *steps) {
    if (!s || !out) return tyee::fail(TYEE_EINVAL, "null argument");
    out[0] = s->ms_edge;
    out[1] = s->ms_face;
    if (steps) *steps = s->timed;
    return TYEE_OK;
}

extern "C" int tyee_tet_sim_destroy(tyee_tet_sim *s) {
    delete s;
    return TYEE_OK;
}
