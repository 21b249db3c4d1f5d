// libtyee device runtime for AMD Instinct MI355X (gfx950): the leap-frog half-step kernels
// of the triangular Yee-like scheme (arXiv:1812.01448, eqs. 3-6) and the simulation
// object behind the C ABI.
//
// Device formulation. Every edge stores the scaled field Et_i = gamma_i |e_i| E_i, which
// turns both half-steps into one coefficient per cell:
//   edge i     : Et_i += cE_i (B_R - B_L),         cE_i = dt gamma_i^2 |e_i| / d_i   (eq. 3)
//   triangle j : B_j  += nB_j sum_q s(j,q) Et_A,   nB_j = -dt / S_j                 (eq. 4)
// Signs s(j,q) live in bit 31 of the edge index; outer edges of a closed resonator have
// cE = 0 and both neighbour slots pointing at their one triangle, so they stay at zero
// without a branch. The plasma current (eq. 5) and the soft source act on a short list of
// "special" edges that a small kernel pre-corrects before the edge half-step (eq. 6).
// Fields, coefficients and indices are separate arrays (structure of arrays) so every
// per-cell access is a coalesced 4- or 8-byte load; only the neighbour gathers are
// indirect, and the locality numbering keeps them inside a small window.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

#include "internal.hpp"
#include "kernels.hpp"
#include "sim.hpp"

namespace tyee {



namespace {

template <typename T> int upload(DeviceBuffer &buf, const std::vector<double> &host, hipStream_t s) {
    std::vector<T> tmp(host.begin(), host.end());
    int rc = buf.alloc(tmp.size() * sizeof(T));
    if (rc) return rc;
    if (tmp.empty()) return TYEE_OK;
    TYEE_HIP(hipMemcpyAsync(buf.p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
    TYEE_HIP(hipStreamSynchronize(s));
    return TYEE_OK;
}

template <typename I> int upload_raw(DeviceBuffer &buf, const std::vector<I> &host, hipStream_t s) {
    int rc = buf.alloc(host.size() * sizeof(I));
    if (rc) return rc;
    if (host.empty()) return TYEE_OK;
    TYEE_HIP(hipMemcpyAsync(buf.p, host.data(), host.size() * sizeof(I), hipMemcpyHostToDevice, s));
    TYEE_HIP(hipStreamSynchronize(s));
    return TYEE_OK;
}

template <typename T> int upload_doubles(Sim &s, DeviceBuffer &buf, const std::vector<double> &host) {
    return upload<T>(buf, host, s.stream);
}

int upload_field(Sim &s, DeviceBuffer &buf, const std::vector<double> &host) {
    return s.f64 ? upload_doubles<double>(s, buf, host) : upload_doubles<float>(s, buf, host);
}

int download_field(Sim &s, const DeviceBuffer &buf, std::vector<double> &host, int64_t n) {
    host.resize(n);
    if (n == 0) return TYEE_OK;
    if (s.f64) {
        TYEE_HIP(hipMemcpyAsync(host.data(), buf.p, n * sizeof(double), hipMemcpyDeviceToHost, s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
    } else {
        std::vector<float> tmp(n);
        TYEE_HIP(hipMemcpyAsync(tmp.data(), buf.p, n * sizeof(float), hipMemcpyDeviceToHost, s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
        std::copy(tmp.begin(), tmp.end(), host.begin());
    }
    return TYEE_OK;
}

// Coefficients of the two half-steps in device numbering (FP64, rounded once on upload).
int upload_coefficients(Sim &s) {
    std::vector<double> ce(s.ne), nb(s.nt);
    for (int64_t k = 0; k < s.ne; ++k) {
        int32_t i = s.perm_e[k];
        bool inner = s.R[i] >= 0 && s.L[i] >= 0;
        ce[k] = inner ? s.dt_edge[i] * s.gamma[i] * s.gamma[i] * s.elen[i] / s.d[i] : 0.0;
    }
    for (int64_t k = 0; k < s.nt; ++k) nb[k] = -s.dt_tri[s.perm_t[k]] / s.S[s.perm_t[k]];
    s.graph_dirty = true;
    s.diag_ready = false;
    s.ce_dev = ce;
    s.nb_dev = nb;
    int rc = upload_field(s, s.cE, ce);
    if (!rc) rc = upload_field(s, s.nB, nb);
    if (!rc && s.tiling) rc = refresh_tiling_coefficients(s);
    return rc;
}

int upload_connectivity(Sim &s) {
    std::vector<int32_t> rl(2 * s.ne), a0(s.nt), a1(s.nt), a2(s.nt);
    for (int64_t k = 0; k < s.ne; ++k) {
        int32_t i = s.perm_e[k];
        int32_t r = s.R[i], l = s.L[i];
        int32_t one = r >= 0 ? r : l;  // outer edge: both slots on its one triangle
        rl[2 * k] = s.slot_t[r >= 0 ? r : one];
        rl[2 * k + 1] = s.slot_t[l >= 0 ? l : one];
    }
    std::vector<int32_t> *dst[3] = {&a0, &a1, &a2};
    for (int64_t k = 0; k < s.nt; ++k) {
        int32_t j = s.perm_t[k];
        for (int q = 0; q < 3; ++q) {
            uint32_t slot = uint32_t(s.slot_e[s.A[3 * j + q]]);
            if (s.sgn[3 * j + q] < 0) slot |= 0x80000000u;
            (*dst[q])[k] = int32_t(slot);
        }
    }
    int rc = upload_raw(s.RL, rl, s.stream);
    if (!rc) rc = upload_raw(s.A0, a0, s.stream);
    if (!rc) rc = upload_raw(s.A1, a1, s.stream);
    if (!rc) rc = upload_raw(s.A2, a2, s.stream);
    return rc;
}

// Special edges: plasma edges (wp2 > 0) and source edges, each listed once.  The nodal
// charge list holds every interior node touching a special edge with its incidences.
int rebuild_specials(Sim &s) {
    std::vector<int64_t> which(s.ne, -1);
    s.sp_edge.clear();
    s.sp_plasma.clear();
    auto add = [&](int32_t i) {
        if (which[i] < 0) {
            which[i] = int64_t(s.sp_edge.size());
            s.sp_edge.push_back(i);
            s.sp_plasma.push_back(0);
        }
        return which[i];
    };
    if (!s.wp2_edge.empty())
        for (int64_t i = 0; i < s.ne; ++i)
            if (s.wp2_edge[i] > 0.0) s.sp_plasma[add(int32_t(i))] = 1;
    std::vector<double> wsum;
    for (size_t r = 0; r < s.src_edge.size(); ++r) add(s.src_edge[r]);
    const int64_t n = int64_t(s.sp_edge.size());
    s.n_special = n;
    std::vector<int32_t> slot(n);
    std::vector<double> ca(n, 0.0), cb(n, 0.0), w(n, 0.0), zero(n, 0.0);
    const double half = s.nu * s.dt / 2.0;
    for (int64_t k = 0; k < n; ++k) {
        int32_t i = s.sp_edge[k];
        slot[k] = s.slot_e[i];
        if (s.sp_plasma[k]) {
            ca[k] = (1.0 - half) / (1.0 + half);
            cb[k] = s.dt * s.wp2_edge[i] / (1.0 + half);
        }
    }
    // Et is decreased by dt * scale * Jsrc = (dt * scale * w) * g(t)
    for (size_t r = 0; r < s.src_edge.size(); ++r) {
        int32_t i = s.src_edge[r];
        w[which[i]] += s.dt * s.scale(i) * s.src_w[r];
    }
    int rc = upload_raw(s.sp_slot, slot, s.stream);
    for (int b = 0; b < 2 && !rc; ++b) rc = upload_field(s, s.sp_j_buf[b], zero);
    if (!rc) rc = upload_field(s, s.sp_ca, ca);
    if (!rc) rc = upload_field(s, s.sp_cb, cb);
    if (!rc) rc = upload_field(s, s.sp_w, w);
    if (!rc) rc = upload_field(s, s.sp_delta, std::vector<double>(size_t(n) * kMaxFusion, 0.0));
    if (rc) return rc;
    // the fused tiles carry each local edge's special-list index: rebuild them lazily
    s.tiling.reset();
    s.graph_dirty = true;

    // node incidences: Q_k -= sum sigma(k,i) d_i/scale_i * delta_i  (delta = dt scale (j + Jsrc))
    std::vector<std::vector<std::pair<int32_t, double>>> inc(s.nv);
    for (int64_t k = 0; k < n; ++k) {
        int32_t i = s.sp_edge[k];
        double c = s.d[i] / s.scale(i);
        int32_t lo = s.edge[2 * i], hi = s.edge[2 * i + 1];
        if (!s.node_outer[lo]) inc[lo].push_back({int32_t(k), +c});
        if (!s.node_outer[hi]) inc[hi].push_back({int32_t(k), -c});
    }
    std::vector<int32_t> qn, off{0}, qk;
    std::vector<double> qc;
    for (int64_t v = 0; v < s.nv; ++v) {
        if (inc[v].empty()) continue;
        qn.push_back(int32_t(v));
        for (auto &p : inc[v]) {
            qk.push_back(p.first);
            qc.push_back(p.second);
        }
        off.push_back(int32_t(qk.size()));
    }
    for (auto &pp : s.probes) {
        if (pp->field != TYEE_FIELD_J) continue;
        std::vector<int32_t> sl(pp->n, 0);
        for (int64_t r = 0; r < pp->n; ++r) sl[r] = which[pp->ids[r]] >= 0 ? int32_t(which[pp->ids[r]]) : 0;
        if ((rc = upload_raw(pp->slots, sl, s.stream))) return rc;
    }
    s.n_qnode = int64_t(qn.size());
    rc = upload_raw(s.q_node, qn, s.stream);
    if (!rc) rc = upload_raw(s.q_off, off, s.stream);
    if (!rc) rc = upload_raw(s.q_inc, qk, s.stream);
    if (!rc) rc = upload_field(s, s.q_coef, qc);
    return rc;
}


// Launch one kernel kind, bracketed by timing events when that kind is profiled.
template <typename F> int timed(Sim &s, int kind, F &&launch) {
    int rc;
    int slot = s.timer.begin(kind, s.stream, &rc);
    if (rc) return rc;
    rc = launch();
    if (rc) return rc;
    return s.timer.end(slot, s.stream);
}

// Device array and slot list a probe reads from.
template <typename T> const T *probe_source(Sim &s, const Probe &p) {
    switch (p.field) {
    case TYEE_FIELD_E: return s.Et().as<T>();
    case TYEE_FIELD_B: return s.B().as<T>();
    case TYEE_FIELD_J: return s.sp_j().as<T>();
    default: return s.Q.as<T>();
    }
}

template <typename T> int sample_probes(Sim &s) {
    for (auto &pp : s.probes) {
        Probe &p = *pp;
        if (s.step % p.every != 0 || p.taken >= p.capacity) continue;
        k_probe<T><<<int((p.n + 255) / 256), 256, 0, s.stream>>>(int(p.n), p.slots.as<int32_t>(),
                                                                 probe_source<T>(s, p),
                                                                 p.samples.as<T>() + p.taken * p.n);
        ++p.taken;
    }
    return TYEE_OK;
}

// Largest step count from s.step that does not cross a probe's sampling step.
int64_t steps_to_next_sample(const Sim &s) {
    int64_t best = INT64_MAX;
    for (auto &p : s.probes)
        if (p->taken < p->capacity) best = std::min(best, p->every - s.step % p->every);
    return best;
}

// Replay `graph_launches` fused launches captured in a HIP graph (captured on first use and
// whenever the tiling, coefficients or buffers changed).  An even launch count returns the
// field buffers to the same parity, so one graph serves every replay.
template <typename T> int replay_graph(Sim &s, int k) {
    if (s.graph_dirty || !s.graph || s.graph_K != k || s.graph_cur != s.cur) {
        if (s.graph) {
            (void)hipGraphExecDestroy(s.graph);
            s.graph = nullptr;
        }
        const int cur0 = s.cur;
        TYEE_HIP(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
        int rc = TYEE_OK;
        if (k > 1) {
            for (int g = 0; g < s.graph_launches && !rc; ++g) rc = launch_fused<T>(s, k);
        } else {  // one step per "launch": the edge and the triangle half-step
            const int ge = blocks_for(s.ne), gt = blocks_for(s.nt);
            for (int g = 0; g < s.graph_launches; ++g) {
                launch_edge<T>(s.stream, s.ne, ge, s.Et().as<T>(), s.B().as<T>(), s.cE.as<T>(), s.RL.as<int2>());
                launch_tri<T>(s.stream, s.nt, gt, s.B().as<T>(), s.Et().as<T>(), s.nB.as<T>(), s.A0.as<uint32_t>(),
                              s.A1.as<uint32_t>(), s.A2.as<uint32_t>());
            }
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s.stream, &graph);
        s.cur = cur0;
        if (rc) return rc;
        if (e != hipSuccess) return fail(TYEE_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&s.graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(TYEE_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        s.graph_dirty = false;
        s.graph_K = k;
        s.graph_cur = s.cur;
    }
    return timed(s, TYEE_KERNEL_GRAPH, [&]() -> int {
        TYEE_HIP(hipGraphLaunch(s.graph, s.stream));
        return TYEE_OK;
    });
}

template <typename T> int enqueue_steps(Sim &s, int64_t n) {
    const int ge = blocks_for(s.ne), gt = blocks_for(s.nt);
    const T *cE = s.cE.as<T>(), *nB = s.nB.as<T>();
    const int2 *RL = s.RL.as<int2>();
    const uint32_t *a0 = s.A0.as<uint32_t>(), *a1 = s.A1.as<uint32_t>(), *a2 = s.A2.as<uint32_t>();
    const bool special = s.n_special > 0;
    int64_t done = 0;
    int rc = TYEE_OK;
    while (done < n && !rc) {
        T *Et = s.Et().as<T>(), *B = s.B().as<T>();
        int k = s.fusion;
        if (k > n - done || k > steps_to_next_sample(s)) k = 1;  // remainder: single steps
        if (special && k == 1) {
            const double g = waveform((double(s.step) + 0.5) * s.dt, s.src_omega, s.src_cycles);
            rc = timed(s, TYEE_KERNEL_SPECIAL, [&] {
                launch_special<T>(s.stream, s.n_special, s.sp_slot.as<int32_t>(), Et, s.sp_j().as<T>(),
                                  s.sp_ca.as<T>(), s.sp_cb.as<T>(), s.sp_w.as<T>(), s.sp_delta.as<T>(),
                                  T(g), T(s.dt));
                return TYEE_OK;
            });
            if (!rc && s.n_qnode > 0)
                rc = timed(s, TYEE_KERNEL_CHARGE, [&] {
                    launch_charge<T>(s.stream, s.n_qnode, s.q_node.as<int32_t>(), s.q_off.as<int32_t>(),
                                     s.q_inc.as<int32_t>(), s.q_coef.as<T>(), s.sp_delta.as<T>(), 1,
                                     int(s.n_special), s.Q.as<T>());
                    return TYEE_OK;
                });
        }
        if (rc) break;
        // graphs replay fixed arguments: the source waveform changes every step, so runs with
        // special edges launch the fused kernel eagerly
        if (!special && s.graph_launches > 0 && k == s.fusion && !s.timer_wants_kernels()) {
            const int64_t span = int64_t(k) * s.graph_launches;
            if (n - done >= span && steps_to_next_sample(s) >= span) {
                if (k > 1 && (!s.tiling || s.tiling->K != k)) {
                    rc = build_tiling(s, k, s.tile_tris);
                    if (rc == TYEE_EINVAL) {  // this mesh does not tile at that depth
                        clear_error();
                        s.fusion = 1;
                        rc = TYEE_OK;
                        continue;
                    }
                    if (rc) break;
                }
                rc = replay_graph<T>(s, k);
                if (rc) break;
                s.step += span;
                done += span;
                if (!s.probes.empty()) rc = sample_probes<T>(s);
                continue;
            }
        }
        if (k > 1 && (!s.tiling || s.tiling->K != k)) {
            rc = build_tiling(s, k, s.tile_tris);
            if (rc == TYEE_EINVAL) {  // this mesh does not tile at that depth: plain launches
                clear_error();
                rc = TYEE_OK;
                s.fusion = 1;
                k = 1;
            }
            if (rc) break;
        }
        if (k > 1) {
            // with special edges this also advances the nodal charge
            rc = timed(s, TYEE_KERNEL_FUSED, [&] { return launch_fused<T>(s, k); });
        } else {
            rc = timed(s, TYEE_KERNEL_EDGE, [&] {
                launch_edge<T>(s.stream, s.ne, ge, Et, B, cE, RL);
                return TYEE_OK;
            });
            if (!rc)
                rc = timed(s, TYEE_KERNEL_TRI, [&] {
                    launch_tri<T>(s.stream, s.nt, gt, B, Et, nB, a0, a1, a2);
                    return TYEE_OK;
                });
        }
        s.step += k;
        done += k;
        if (!rc && !s.probes.empty()) rc = sample_probes<T>(s);
    }
    if (rc) return rc;
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

}  // namespace

Sim::~Sim() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    probes.clear();
    tiling.reset();
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// Set up a simulation of mesh m: copies of the host arrays it needs, zero fields, packed
// coefficients and connectivity on the device.  dt_tri / dt_edge: time step per canonical
// triangle / edge.
int init_sim(Sim &s, const Mesh &m, int32_t prec, const std::vector<double> &dt_tri,
             const std::vector<double> &dt_edge, void *stream) {
    s.f64 = prec == TYEE_F64;
    s.esz = s.f64 ? 8 : 4;
    s.dt = dt_tri.empty() ? 0.0 : dt_tri[0];
    s.dt_tri = dt_tri;
    s.dt_edge = dt_edge;
    s.nv = m.nv;
    s.ne = m.ne;
    s.nt = m.nt;
    s.perm_t = m.perm_t;
    s.perm_e = m.perm_e;
    s.slot_t.resize(m.nt);
    s.slot_e.resize(m.ne);
    for (int64_t k = 0; k < m.nt; ++k) s.slot_t[m.perm_t[k]] = int32_t(k);
    for (int64_t k = 0; k < m.ne; ++k) s.slot_e[m.perm_e[k]] = int32_t(k);
    s.edge = m.edge;
    s.R = m.R;
    s.L = m.L;
    s.A = m.A;
    s.sgn = m.sgn;
    s.elen = m.elen;
    s.d = m.d;
    s.hR = m.hR;
    s.hL = m.hL;
    s.S = m.S;
    s.node_outer = m.node_outer;
    s.gamma.assign(m.ne, 1.0);
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return fail(TYEE_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
    s.device = device;
    if (stream) {
        s.stream = static_cast<hipStream_t>(stream);
    } else {
        // graphs cannot be captured on the legacy default stream: use a stream of our own
        TYEE_HIP(hipStreamCreate(&s.stream));
        s.own_stream = true;
    }
    std::vector<double> zero_e(m.ne, 0.0), zero_t(m.nt, 0.0), zero_v(m.nv, 0.0);
    int rc = TYEE_OK;
    for (int b = 0; b < 2 && !rc; ++b) {
        rc = upload_field(s, s.Et_buf[b], zero_e);
        if (!rc) rc = upload_field(s, s.B_buf[b], zero_t);
    }
    if (!rc) rc = upload_field(s, s.Q, zero_v);
    if (!rc) rc = upload_coefficients(s);
    if (!rc) rc = upload_connectivity(s);
    if (!rc) rc = rebuild_specials(s);
    if (rc) return rc;
    if (hipEventCreate(&s.ev0) != hipSuccess || hipEventCreate(&s.ev1) != hipSuccess)
        return fail(TYEE_EDEVICE, "hipEventCreate failed");
    return TYEE_OK;
}

namespace {

// FP64 tables of the diagnostics reduction, in device numbering.
int build_diag_tables(Sim &s) {
    std::vector<double> wE(s.ne), S(s.nt), dtS(s.nt);
    std::vector<float> inv(s.ne);
    for (int64_t k = 0; k < s.ne; ++k) {
        const int32_t i = s.perm_e[k];
        const bool inner = s.R[i] >= 0 && s.L[i] >= 0;
        wE[k] = inner ? s.d[i] / (s.gamma[i] * s.gamma[i] * s.elen[i]) : 0.0;
        inv[k] = float(1.0 / s.scale(i));
    }
    for (int64_t k = 0; k < s.nt; ++k) {
        const int32_t j = s.perm_t[k];
        S[k] = s.S[j];
        dtS[k] = s.dt_tri[j] / s.S[j];
    }
    int rc = upload<double>(s.diag_wE, wE, s.stream);
    if (!rc) rc = upload_raw(s.diag_inv_scale, inv, s.stream);
    if (!rc) rc = upload<double>(s.diag_S, S, s.stream);
    if (!rc) rc = upload<double>(s.diag_dtS, dtS, s.stream);
    const size_t nblocks = size_t((std::max(s.ne, s.nt) + kDiagThreads - 1) / kDiagThreads);
    if (!rc) rc = s.diag_partial.alloc(size_t(6) * std::max<size_t>(1, nblocks) * sizeof(double));
    if (!rc) s.diag_ready = true;
    return rc;
}

template <typename T> int device_diagnostics(Sim &s, double *sums) {
    const int64_t n = std::max(s.ne, s.nt);
    const int nb = int((n + kDiagThreads - 1) / kDiagThreads);
    k_diag<T><<<nb, kDiagThreads, 0, s.stream>>>(int(s.ne), int(s.nt), s.Et().as<T>(), s.B().as<T>(),
                                                 s.A0.as<uint32_t>(), s.A1.as<uint32_t>(), s.A2.as<uint32_t>(),
                                                 s.diag_wE.as<double>(), s.diag_inv_scale.as<float>(),
                                                 s.diag_S.as<double>(), s.diag_dtS.as<double>(),
                                                 s.diag_partial.as<double>());
    TYEE_HIP(hipGetLastError());
    std::vector<double> part(size_t(6) * nb);
    TYEE_HIP(hipMemcpyAsync(part.data(), s.diag_partial.p, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                            s.stream));
    TYEE_HIP(hipStreamSynchronize(s.stream));
    for (int q = 0; q < 6; ++q) sums[q] = 0.0;
    for (int b = 0; b < nb; ++b) {
        sums[0] += part[6 * size_t(b)];
        sums[1] += part[6 * size_t(b) + 1];
        sums[2] += part[6 * size_t(b) + 2];
        sums[3] = std::max(sums[3], part[6 * size_t(b) + 3]);
        sums[4] = std::max(sums[4], part[6 * size_t(b) + 4]);
        sums[5] += part[6 * size_t(b) + 5];
    }
    return TYEE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Diagnostics without allocation: the per-block partial sums of k_diag and their six totals
// live in a fixed device array instead of a buffer the simulation allocates.
// ---------------------------------------------------------------------------------------

// k_diag blocks the array holds: meshes with up to kDiagStaticBlocks * kDiagThreads
// (33,554,432) edges and as many triangles.
constexpr int64_t kDiagStaticBlocks = 131072;
constexpr size_t kDiagStaticTotals = size_t(6) * kDiagStaticBlocks;  // offset of the six totals

// 6.0 MiB per device, held until the process ends; every call on a device shares it.
static __device__ __align__(256) double scratch[6 * kDiagStaticBlocks + 8];

// The six totals of nb per-block partials, each column added in block order with the same
// operations as the host loop of device_diagnostics (so both entry points agree bit for bit).
__global__ __launch_bounds__(64) void k_diag_total(int nb, double *__restrict__ buf) {
    const int q = threadIdx.x;
    if (q >= 6) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double v = buf[6 * size_t(b) + q];
        if (q == 3 || q == 4) acc = acc < v ? v : acc;
        else acc += v;
    }
    buf[kDiagStaticTotals + q] = acc;
}

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int static_scratch(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return fail(TYEE_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TYEE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return TYEE_OK;
}

// Makes `device` current for the lifetime of the guard, restoring the previous one.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int device) {
        int cur = 0;
        err = hipGetDevice(&cur);
        if (err == hipSuccess && cur != device) {
            err = hipSetDevice(device);
            if (err == hipSuccess) prev = cur;
        }
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T> int device_diagnostics_static(Sim &s, double *buf, double *sums) {
    const int64_t n = std::max(s.ne, s.nt);
    const int nb = int((n + kDiagThreads - 1) / kDiagThreads);
    k_diag<T><<<nb, kDiagThreads, 0, s.stream>>>(int(s.ne), int(s.nt), s.Et().as<T>(), s.B().as<T>(),
                                                 s.A0.as<uint32_t>(), s.A1.as<uint32_t>(), s.A2.as<uint32_t>(),
                                                 s.diag_wE.as<double>(), s.diag_inv_scale.as<float>(),
                                                 s.diag_S.as<double>(), s.diag_dtS.as<double>(), buf);
    TYEE_HIP(hipGetLastError());
    k_diag_total<<<1, 64, 0, s.stream>>>(nb, buf);
    TYEE_HIP(hipGetLastError());
    TYEE_HIP(hipMemcpyAsync(sums, buf + kDiagStaticTotals, 6 * sizeof(double), hipMemcpyDeviceToHost, s.stream));
    TYEE_HIP(hipStreamSynchronize(s.stream));
    return TYEE_OK;
}

}  // namespace

// Device copy-rate probe: one 16-byte element per work-item, non-temporal loads and stores
// (streaming data that is not reused), the form that reaches the highest copy rate.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy_probe(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                    int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace tyee

// ---------------------------------------------------------------------------------------
// C ABI: simulation
// ---------------------------------------------------------------------------------------


using tyee::fail;

extern "C" {

int tyee_sim_create(const tyee_mesh *mesh, int32_t prec, double dt, void *stream, tyee_sim **out) {
    if (!mesh || !out) return fail(TYEE_EINVAL, "null argument");
    *out = nullptr;
    if (prec != TYEE_F32 && prec != TYEE_F64) return fail(TYEE_EINVAL, "prec must be TYEE_F32 or TYEE_F64");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(TYEE_EINVAL, "dt must be positive and finite");
    try {
        std::unique_ptr<tyee_sim> h(new tyee_sim());
        const tyee::Mesh &m = mesh->m;
        int rc = tyee::init_sim(h->s, m, prec, std::vector<double>(m.nt, dt), std::vector<double>(m.ne, dt),
                                stream);
        if (rc) return rc;
        *out = h.release();
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

int tyee_sim_set_state(tyee_sim *sim, int32_t field, const double *host) {
    if (!sim || !host) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    std::vector<double> dev;
    switch (field) {
    case TYEE_FIELD_E:
        dev.resize(s.ne);
        for (int64_t k = 0; k < s.ne; ++k) {
            int32_t i = s.perm_e[k];
            dev[k] = (s.R[i] >= 0 && s.L[i] >= 0) ? s.scale(i) * host[i] : 0.0;
        }
        return tyee::upload_field(s, s.Et(), dev);
    case TYEE_FIELD_B:
        dev.resize(s.nt);
        for (int64_t k = 0; k < s.nt; ++k) dev[k] = host[s.perm_t[k]];
        return tyee::upload_field(s, s.B(), dev);
    case TYEE_FIELD_J: {
        std::vector<uint8_t> listed(s.ne, 0);
        dev.assign(s.n_special, 0.0);
        for (int64_t k = 0; k < s.n_special; ++k)
            if (s.sp_plasma[k]) {
                int32_t i = s.sp_edge[k];
                listed[i] = 1;
                dev[k] = s.scale(i) * host[i];
            }
        for (int64_t i = 0; i < s.ne; ++i)
            if (!listed[i] && host[i] != 0.0) return fail(TYEE_EINVAL, "current on a non-plasma edge");
        if (s.n_special == 0) return TYEE_OK;
        return tyee::upload_field(s, s.sp_j(), dev);
    }
    case TYEE_FIELD_Q:
        dev.assign(host, host + s.nv);
        return tyee::upload_field(s, s.Q, dev);
    default:
        return fail(TYEE_EINVAL, "unknown field");
    }
}

int tyee_sim_get_state(tyee_sim *sim, int32_t field, double *host) {
    if (!sim || !host) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    std::vector<double> dev;
    int rc;
    switch (field) {
    case TYEE_FIELD_E:
        if ((rc = tyee::download_field(s, s.Et(), dev, s.ne))) return rc;
        for (int64_t k = 0; k < s.ne; ++k) {
            int32_t i = s.perm_e[k];
            host[i] = dev[k] / s.scale(i);
        }
        return TYEE_OK;
    case TYEE_FIELD_B:
        if ((rc = tyee::download_field(s, s.B(), dev, s.nt))) return rc;
        for (int64_t k = 0; k < s.nt; ++k) host[s.perm_t[k]] = dev[k];
        return TYEE_OK;
    case TYEE_FIELD_J:
        std::fill(host, host + s.ne, 0.0);
        if (s.n_special == 0) return TYEE_OK;
        if ((rc = tyee::download_field(s, s.sp_j(), dev, s.n_special))) return rc;
        for (int64_t k = 0; k < s.n_special; ++k)
            if (s.sp_plasma[k]) host[s.sp_edge[k]] = dev[k] / s.scale(s.sp_edge[k]);
        return TYEE_OK;
    case TYEE_FIELD_Q:
        if ((rc = tyee::download_field(s, s.Q, dev, s.nv))) return rc;
        std::copy(dev.begin(), dev.end(), host);
        return TYEE_OK;
    default:
        return fail(TYEE_EINVAL, "unknown field");
    }
}

int tyee_sim_set_media(tyee_sim *sim, const double *wp2_tri, double nu) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    if (!(nu >= 0.0) || !std::isfinite(nu)) return fail(TYEE_EINVAL, "nu must be >= 0");
    tyee::Sim &s = sim->s;
    if (!wp2_tri) {
        s.wp2_edge.clear();
        s.nu = 0.0;
        return tyee::rebuild_specials(s);
    }
    for (int64_t j = 0; j < s.nt; ++j)
        if (!(wp2_tri[j] >= 0.0) || !std::isfinite(wp2_tri[j]))
            return fail(TYEE_EINVAL, "plasma frequency squared must be finite and >= 0");
    s.wp2_edge.assign(s.ne, 0.0);
    for (int64_t i = 0; i < s.ne; ++i)
        if (s.R[i] >= 0 && s.L[i] >= 0)
            s.wp2_edge[i] = (s.hR[i] * wp2_tri[s.R[i]] + s.hL[i] * wp2_tri[s.L[i]]) / s.d[i];
    s.nu = nu;
    return tyee::rebuild_specials(s);
}

int tyee_sim_set_source(tyee_sim *sim, const int32_t *pairs, const double *weights, int64_t n,
                        double omega, double cycles) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    tyee::Sim &s = sim->s;
    if (n < 0 || (n > 0 && (!pairs || !weights))) return fail(TYEE_EINVAL, "bad source arrays");
    if (n > 0 && (!(omega > 0.0) || !(cycles > 0.0))) return fail(TYEE_EINVAL, "omega, cycles must be > 0");
    std::vector<int32_t> ids(n);
    std::vector<double> w(n);
    for (int64_t r = 0; r < n; ++r) {
        int32_t a = pairs[2 * r], b = pairs[2 * r + 1];
        if (a < 0 || b < 0 || a >= s.nv || b >= s.nv || a == b) return fail(TYEE_EINVAL, "bad node pair");
        int32_t lo = std::min(a, b), hi = std::max(a, b);
        // edges are sorted by (lo, hi): binary search
        int64_t left = 0, right = s.ne;
        while (left < right) {
            int64_t mid = (left + right) / 2;
            int32_t ml = s.edge[2 * mid], mh = s.edge[2 * mid + 1];
            if (ml < lo || (ml == lo && mh < hi)) left = mid + 1;
            else right = mid;
        }
        if (left >= s.ne || s.edge[2 * left] != lo || s.edge[2 * left + 1] != hi)
            return fail(TYEE_EINVAL, "node pair is not a mesh edge");
        if (!(s.R[left] >= 0 && s.L[left] >= 0)) return fail(TYEE_EINVAL, "source on an outer edge");
        ids[r] = int32_t(left);
        w[r] = a < b ? weights[r] : -weights[r];
    }
    s.src_edge = ids;
    s.src_w = w;
    s.src_omega = n > 0 ? omega : 1.0;
    s.src_cycles = n > 0 ? cycles : 1.0;
    // keep the plasma current across a source change
    std::vector<double> J(s.ne, 0.0);
    int rc = tyee_sim_get_state(sim, TYEE_FIELD_J, J.data());
    if (!rc) rc = tyee::rebuild_specials(s);
    if (!rc) rc = tyee_sim_set_state(sim, TYEE_FIELD_J, J.data());
    return rc;
}

int tyee_sim_set_edge_scale(tyee_sim *sim, const double *gamma) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    tyee::Sim &s = sim->s;
    if (gamma)
        for (int64_t i = 0; i < s.ne; ++i)
            if (!(gamma[i] > 0.0) || !std::isfinite(gamma[i])) return fail(TYEE_EINVAL, "gamma must be > 0");
    std::vector<double> E(s.ne), J(s.ne);
    int rc = tyee_sim_get_state(sim, TYEE_FIELD_E, E.data());
    if (!rc) rc = tyee_sim_get_state(sim, TYEE_FIELD_J, J.data());
    if (rc) return rc;
    if (gamma) s.gamma.assign(gamma, gamma + s.ne);
    else s.gamma.assign(s.ne, 1.0);
    rc = tyee::upload_coefficients(s);
    if (!rc) rc = tyee::rebuild_specials(s);
    if (!rc) rc = tyee_sim_set_state(sim, TYEE_FIELD_E, E.data());
    if (!rc) rc = tyee_sim_set_state(sim, TYEE_FIELD_J, J.data());
    return rc;
}

int tyee_sim_set_fusion(tyee_sim *sim, int32_t k, int32_t tile_tris) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    // default depth in FP32: 6 steps per launch on 1536-triangle tiles (4M triangles: 9.5
    // against 10.7 us per step at 4 steps); meshes of 8M triangles or more, whose fields no
    // longer fit the Infinity Cache, take 8 on 1024-triangle tiles (16M triangles: 48.8 us per
    // step; 6 and 7 steps are within 2.3 %, 4 steps 61.2).  FP64 keeps 4.
    if (k == 0) k = sim->s.f64 ? 4 : (sim->s.nt >= 8000000 ? 8 : 6);
    if (k < 1 || k > tyee::kMaxFusion) return fail(TYEE_EINVAL, "steps per launch must be 0 (default) or 1..8");
    if (tile_tris != 0 && (tile_tris < 256 || tile_tris > 8192))
        return fail(TYEE_EINVAL, "tile size must be 0 or in [256, 8192] triangles");
    tyee::Sim &s = sim->s;
    if (s.tile_tris != tile_tris) s.tiling.reset();
    s.fusion = k;
    s.tile_tris = tile_tris;
    s.graph_dirty = true;
    return TYEE_OK;
}

int tyee_sim_set_graph(tyee_sim *sim, int32_t launches) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    if (launches < 0 || launches % 2 || launches > 1024)
        return fail(TYEE_EINVAL, "launches per graph must be 0 or an even number up to 1024");
    sim->s.graph_launches = launches;
    sim->s.graph_dirty = true;
    return TYEE_OK;
}

int tyee_sim_step(tyee_sim *sim, int64_t n) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    if (n < 0) return fail(TYEE_EINVAL, "negative step count");
    tyee::Sim &s = sim->s;
    if (n == 0) return TYEE_OK;
    TYEE_HIP(hipEventRecord(s.ev0, s.stream));
    int rc = s.f64 ? tyee::enqueue_steps<double>(s, n) : tyee::enqueue_steps<float>(s, n);
    if (rc) return rc;
    TYEE_HIP(hipEventRecord(s.ev1, s.stream));
    return TYEE_OK;
}

int tyee_sim_sync(tyee_sim *sim) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    TYEE_HIP(hipStreamSynchronize(sim->s.stream));
    return TYEE_OK;
}

int tyee_sim_last_step_ms(tyee_sim *sim, double *ms) {
    if (!sim || !ms) return fail(TYEE_EINVAL, "null argument");
    TYEE_HIP(hipEventSynchronize(sim->s.ev1));
    float f = 0.0f;
    TYEE_HIP(hipEventElapsedTime(&f, sim->s.ev0, sim->s.ev1));
    *ms = f;
    return TYEE_OK;
}


int tyee_sim_diagnostics(tyee_sim *sim, tyee_diag *out) {
    if (!sim || !out) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    int rc = TYEE_OK;
    if (!s.diag_ready) rc = tyee::build_diag_tables(s);
    if (rc) return rc;
    if (int64_t(std::max(s.ne, s.nt)) >= int64_t(INT32_MAX)) return fail(TYEE_EINVAL, "mesh too large");
    double v[6];
    rc = s.f64 ? tyee::device_diagnostics<double>(s, v) : tyee::device_diagnostics<float>(s, v);
    if (rc) return rc;
    tyee_diag d{};
    d.step = s.step;
    d.time = double(s.step) * s.dt;
    d.energy = v[0] + v[1];
    d.energy_h = v[0] + v[2];
    d.max_abs_E = v[3];
    d.max_abs_B = v[4];
    d.nonfinite = v[5] > 0.0;
    *out = d;
    return d.nonfinite ? fail(TYEE_EUNSTABLE, "non-finite field value") : TYEE_OK;
}

int tyee_sim_diagnostics_noalloc(tyee_sim *sim, tyee_diag *out) {
    if (!sim || !out) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    if (!s.diag_ready)
        return fail(TYEE_EINVAL, "diagnostics tables are not built: call tyee_sim_diagnostics once after "
                                 "creating the simulation or changing its coefficients");
    if (std::max(s.ne, s.nt) > tyee::kDiagStaticBlocks * tyee::kDiagThreads)
        return fail(TYEE_EINVAL, "mesh too large for the fixed diagnostics scratch (at most 33,554,432 edges "
                                 "and 33,554,432 triangles)");
    tyee::DeviceGuard guard(s.device);
    if (guard.err != hipSuccess)
        return fail(TYEE_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(guard.err));
    double *buf = nullptr;
    int rc = tyee::static_scratch(s.device, &buf);
    if (rc) return rc;
    double v[6];
    rc = s.f64 ? tyee::device_diagnostics_static<double>(s, buf, v)
               : tyee::device_diagnostics_static<float>(s, buf, v);
    if (rc) return rc;
    tyee_diag d{};
    d.step = s.step;
    d.time = double(s.step) * s.dt;
    d.energy = v[0] + v[1];
    d.energy_h = v[0] + v[2];
    d.max_abs_E = v[3];
    d.max_abs_B = v[4];
    d.nonfinite = v[5] > 0.0;
    *out = d;
    return d.nonfinite ? fail(TYEE_EUNSTABLE, "non-finite field value") : TYEE_OK;
}

int tyee_sim_set_profiling(tyee_sim *sim, uint32_t kinds) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    int rc = sim->s.timer.drain();
    if (rc) return rc;
    sim->s.timer.reset(kinds);
    return TYEE_OK;
}

int tyee_sim_kernel_times(tyee_sim *sim, int32_t kind, int64_t *count, double *total_ms) {
    if (!sim || !count || !total_ms) return fail(TYEE_EINVAL, "null argument");
    if (kind < 0 || kind >= tyee::LaunchTimer::kKinds) return fail(TYEE_EINVAL, "unknown kernel kind");
    int rc = sim->s.timer.drain();
    if (rc) return rc;
    *count = sim->s.timer.count[kind];
    *total_ms = sim->s.timer.total_ms[kind];
    return TYEE_OK;
}

int tyee_sim_get_fusion(const tyee_sim *sim, int64_t out[6]) {
    if (!sim || !out) return fail(TYEE_EINVAL, "null argument");
    const tyee::Sim &s = sim->s;
    out[0] = s.fusion;
    const bool built = s.tiling && s.tiling->K == s.fusion;
    out[1] = built ? s.tiling->tile : 0;
    out[2] = built ? s.tiling->ntiles : 0;
    out[3] = built ? s.tiling->sumT : 0;
    out[4] = built ? s.tiling->sumE : 0;
    out[5] = built ? s.tiling->n_sp_tiles : 0;
    return TYEE_OK;
}

int tyee_copy_bandwidth(int64_t bytes, int32_t reps, double *gbs) {
    if (!gbs || bytes < (int64_t(1) << 20) || bytes > (int64_t(1) << 34) || reps < 1 || reps > 1000)
        return fail(TYEE_EINVAL, "bytes must be in [1 MiB, 16 GiB] and reps in [1, 1000]");
    const int64_t n = bytes / 16;
    tyee::DeviceBuffer a, b;
    int rc = a.alloc(size_t(n) * 16);
    if (!rc) rc = b.alloc(size_t(n) * 16);
    if (rc) return rc;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TYEE_HIP(hipStreamCreate(&st));
    auto done = [&](int code) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
        return code;
    };
    if (hipMemsetAsync(a.p, 0, size_t(n) * 16, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        return done(fail(TYEE_EDEVICE, "copy probe set-up failed"));
    const int64_t blocks = (n + 255) / 256;
    const tyee::f32x4 *src = a.as<tyee::f32x4>();
    tyee::f32x4 *dst = b.as<tyee::f32x4>();
    tyee::k_copy_probe<<<dim3(unsigned(blocks)), 256, 0, st>>>(src, dst, n);  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) tyee::k_copy_probe<<<dim3(unsigned(blocks)), 256, 0, st>>>(src, dst, n);
    (void)hipEventRecord(e1, st);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return done(fail(TYEE_EDEVICE, "copy probe launch failed"));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *gbs = 2.0 * double(n) * 16.0 * reps / (double(ms) * 1e-3) / 1e9;
    return done(TYEE_OK);
}

int tyee_sim_bind_external(tyee_sim *sim, int32_t field, void *buf0, void *buf1) {
    if (!sim) return fail(TYEE_EINVAL, "null sim");
    if (field != TYEE_FIELD_E && field != TYEE_FIELD_B) return fail(TYEE_EINVAL, "only E and B can be bound");
    if ((buf0 == nullptr) != (buf1 == nullptr)) return fail(TYEE_EINVAL, "give both buffers or neither");
    tyee::Sim &s = sim->s;
    tyee::DeviceBuffer *buf = field == TYEE_FIELD_E ? s.Et_buf : s.B_buf;
    const size_t n = size_t(field == TYEE_FIELD_E ? s.ne : s.nt) * s.esz;
    void *ext[2] = {buf0, buf1};
    if (buf0) {
        if (buf0 == buf1) return fail(TYEE_EINVAL, "the two buffers must differ");
        for (void *e : ext)
            if (reinterpret_cast<uintptr_t>(e) % s.esz) return fail(TYEE_EINVAL, "misaligned buffer");
        // the current state moves into the caller's buffer of the same parity
        if (n) TYEE_HIP(hipMemcpyAsync(ext[s.cur], buf[s.cur].p, n, hipMemcpyDeviceToDevice, s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
        for (int b = 0; b < 2; ++b) buf[b].borrow(ext[b], n);
    } else {
        if (buf[0].owned) return TYEE_OK;  // nothing bound
        void *own[2] = {nullptr, nullptr};
        for (int b = 0; b < 2; ++b)
            if (n && hipMalloc(&own[b], n) != hipSuccess) {
                if (own[0]) (void)hipFree(own[0]);
                return fail(TYEE_ENOMEM, "hipMalloc failed");
            }
        if (n) TYEE_HIP(hipMemcpyAsync(own[s.cur], buf[s.cur].p, n, hipMemcpyDeviceToDevice, s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
        for (int b = 0; b < 2; ++b) buf[b].adopt(own[b], n);
    }
    s.graph_dirty = true;  // graphs hold buffer addresses
    return TYEE_OK;
}

int tyee_sim_current_buffer(const tyee_sim *sim, int32_t *which) {
    if (!sim || !which) return fail(TYEE_EINVAL, "null argument");
    *which = sim->s.cur;
    return TYEE_OK;
}

int tyee_sim_gauss(tyee_sim *sim, double *out) {
    if (!sim || !out) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    std::vector<double> E(s.ne), Q(s.nv);
    int rc = tyee_sim_get_state(sim, TYEE_FIELD_E, E.data());
    if (!rc) rc = tyee_sim_get_state(sim, TYEE_FIELD_Q, Q.data());
    if (rc) return rc;
    std::fill(out, out + s.nv, 0.0);
    for (int64_t i = 0; i < s.ne; ++i) {
        out[s.edge[2 * i]] += s.d[i] * E[i];
        out[s.edge[2 * i + 1]] -= s.d[i] * E[i];
    }
    for (int64_t v = 0; v < s.nv; ++v) out[v] -= Q[v];
    return TYEE_OK;
}

int tyee_sim_add_probe(tyee_sim *sim, int32_t field, const int32_t *ids, int64_t n, int64_t every,
                       int64_t max_samples, int32_t *probe) {
    if (!sim || !ids || !probe) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    if (n <= 0 || every <= 0 || max_samples <= 0) return fail(TYEE_EINVAL, "n, every, max_samples must be > 0");
    const int64_t limit = field == TYEE_FIELD_B ? s.nt : field == TYEE_FIELD_Q ? s.nv : s.ne;
    if (field < TYEE_FIELD_E || field > TYEE_FIELD_Q) return fail(TYEE_EINVAL, "unknown field");
    auto p = std::make_unique<tyee::Probe>();
    p->field = field;
    p->n = n;
    p->every = every;
    p->capacity = max_samples;
    p->ids.assign(ids, ids + n);
    std::vector<int32_t> sl(n);
    std::vector<int64_t> which(field == TYEE_FIELD_J ? s.ne : 0, -1);
    for (int64_t k = 0; k < s.n_special && field == TYEE_FIELD_J; ++k)
        if (s.sp_plasma[k]) which[s.sp_edge[k]] = k;
    for (int64_t r = 0; r < n; ++r) {
        const int32_t id = ids[r];
        if (id < 0 || id >= limit) return fail(TYEE_EINVAL, "probe id out of range");
        switch (field) {
        case TYEE_FIELD_E: sl[r] = s.slot_e[id]; break;
        case TYEE_FIELD_B: sl[r] = s.slot_t[id]; break;
        case TYEE_FIELD_J:
            if (which[id] < 0) return fail(TYEE_EINVAL, "current probe on a non-plasma edge");
            sl[r] = int32_t(which[id]);
            break;
        default: sl[r] = id;
        }
    }
    int rc = tyee::upload_raw(p->slots, sl, s.stream);
    if (!rc) rc = p->samples.alloc(size_t(n) * size_t(max_samples) * s.esz);
    if (rc) return rc;
    *probe = int32_t(s.probes.size());
    s.probes.push_back(std::move(p));
    return TYEE_OK;
}

int tyee_sim_read_probe(tyee_sim *sim, int32_t probe, double *out, int64_t capacity, int64_t *n_samples) {
    if (!sim || !out || !n_samples) return fail(TYEE_EINVAL, "null argument");
    tyee::Sim &s = sim->s;
    if (probe < 0 || probe >= int32_t(s.probes.size())) return fail(TYEE_EINVAL, "unknown probe");
    tyee::Probe &p = *s.probes[probe];
    const int64_t m = std::min(capacity, p.taken);
    std::vector<double> raw;
    int rc = tyee::download_field(s, p.samples, raw, m * p.n);
    if (rc) return rc;
    for (int64_t t = 0; t < m; ++t)
        for (int64_t r = 0; r < p.n; ++r) {
            double v = raw[t * p.n + r];
            if (p.field == TYEE_FIELD_E || p.field == TYEE_FIELD_J) v /= s.scale(p.ids[r]);
            out[t * p.n + r] = v;
        }
    *n_samples = p.taken;
    return TYEE_OK;
}

int64_t tyee_sim_steps(const tyee_sim *sim) { return sim ? sim->s.step : -1; }

void tyee_sim_destroy(tyee_sim *sim) { delete sim; }

}  // extern "C"
