// Batched stepping of many independent meshes of uneven size.
//
// The members are stored as one disjoint union: their cells are concatenated in the device
// numbering (each member keeps its own locality order inside its range), and each member's
// time step is folded into its cells' coefficients.  One launch of the half-step kernels, or
// of the fused tile kernel, then advances every member at once: tiles are cut from the
// concatenated numbering, so the work list is balanced by construction (equal-sized tiles,
// a tile may straddle two members) and small members cost no extra launches.  A member's
// per-cell arithmetic is exactly that of a standalone simulation with the same time step,
// so every member is bit-identical to its own run.
//
// The autotuner times short trial runs over ordering x steps per launch x tile size with
// HIP events and keeps the fastest; the fields are saved before and restored after.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>

#include "internal.hpp"
#include "sim.hpp"

namespace tyee {
namespace {

int upload_slice(Sim &s, DeviceBuffer &buf, int64_t offset, const std::vector<double> &v) {
    if (v.empty()) return TYEE_OK;
    if (s.f64) {
        TYEE_HIP(hipMemcpyAsync(buf.as<double>() + offset, v.data(), v.size() * sizeof(double),
                                hipMemcpyHostToDevice, s.stream));
    } else {
        std::vector<float> f(v.begin(), v.end());
        TYEE_HIP(hipMemcpyAsync(buf.as<float>() + offset, f.data(), f.size() * sizeof(float),
                                hipMemcpyHostToDevice, s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
        return TYEE_OK;
    }
    TYEE_HIP(hipStreamSynchronize(s.stream));
    return TYEE_OK;
}

int download_slice(Sim &s, const DeviceBuffer &buf, int64_t offset, int64_t n, std::vector<double> &v) {
    v.resize(n);
    if (n == 0) return TYEE_OK;
    if (s.f64) {
        TYEE_HIP(hipMemcpyAsync(v.data(), buf.as<double>() + offset, n * sizeof(double), hipMemcpyDeviceToHost,
                                s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
    } else {
        std::vector<float> f(n);
        TYEE_HIP(hipMemcpyAsync(f.data(), buf.as<float>() + offset, n * sizeof(float), hipMemcpyDeviceToHost,
                                s.stream));
        TYEE_HIP(hipStreamSynchronize(s.stream));
        std::copy(f.begin(), f.end(), v.begin());
    }
    return TYEE_OK;
}

}  // namespace
}  // namespace tyee

struct tyee_batch {
    std::vector<tyee::Mesh> members;
    std::vector<double> dt;
    int32_t prec = TYEE_F32;
    void *stream = nullptr;
    tyee::Mesh merged;
    std::vector<int64_t> off_t, off_e;  // member ranges (canonical = device ranges)
    std::unique_ptr<tyee_sim> sim;
    int32_t fusion = 1, tile = 0, graph = 0;
};

using tyee::fail;

namespace {

// (Re)build the union and its simulation; fields restart at zero.
int rebuild(tyee_batch &b) {
    std::vector<const tyee::Mesh *> parts;
    for (auto &m : b.members) parts.push_back(&m);
    int rc = tyee::merge_meshes(parts, b.merged);
    if (rc) return rc;
    std::vector<double> dt_t, dt_e;
    dt_t.reserve(b.merged.nt);
    dt_e.reserve(b.merged.ne);
    for (size_t p = 0; p < b.members.size(); ++p) {
        dt_t.insert(dt_t.end(), b.members[p].nt, b.dt[p]);
        dt_e.insert(dt_e.end(), b.members[p].ne, b.dt[p]);
    }
    // release the old device state before allocating the new one
    void *stream = b.sim ? (b.sim->s.own_stream ? nullptr : b.sim->s.stream) : b.stream;
    b.sim.reset();
    std::unique_ptr<tyee_sim> h(new tyee_sim());
    rc = tyee::init_sim(h->s, b.merged, b.prec, dt_t, dt_e, stream);
    if (rc) return rc;
    h->s.fusion = b.fusion;
    h->s.tile_tris = b.tile;
    h->s.graph_launches = b.graph;
    b.sim = std::move(h);
    return TYEE_OK;
}

bool member_ok(const tyee_batch *b, int64_t k) { return b && k >= 0 && k < int64_t(b->members.size()); }

// Whole-batch fields in device numbering (host copies), for the tuner's save/restore.
int save_fields(tyee_batch &b, std::vector<double> &E, std::vector<double> &B) {
    tyee::Sim &s = b.sim->s;
    int rc = tyee::download_slice(s, s.Et(), 0, s.ne, E);
    return rc ? rc : tyee::download_slice(s, s.B(), 0, s.nt, B);
}

}  // namespace

extern "C" {

int tyee_batch_create(const tyee_mesh *const *meshes, const double *dt, int64_t n_meshes, int32_t prec,
                      void *stream, tyee_batch **out) {
    if (!meshes || !dt || !out || n_meshes <= 0) return fail(TYEE_EINVAL, "bad batch arguments");
    *out = nullptr;
    if (prec != TYEE_F32 && prec != TYEE_F64) return fail(TYEE_EINVAL, "prec must be TYEE_F32 or TYEE_F64");
    try {
        std::unique_ptr<tyee_batch> b(new tyee_batch());
        b->prec = prec;
        b->stream = stream;
        for (int64_t k = 0; k < n_meshes; ++k) {
            if (!meshes[k]) return fail(TYEE_EINVAL, "null mesh in batch");
            if (!(dt[k] > 0.0) || !std::isfinite(dt[k])) return fail(TYEE_EINVAL, "dt must be positive and finite");
            b->members.push_back(meshes[k]->m);
            b->dt.push_back(dt[k]);
        }
        b->off_t.assign(1, 0);
        b->off_e.assign(1, 0);
        for (auto &m : b->members) {
            b->off_t.push_back(b->off_t.back() + m.nt);
            b->off_e.push_back(b->off_e.back() + m.ne);
        }
        int rc = rebuild(*b);
        if (rc) return rc;
        *out = b.release();
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

int tyee_batch_sim(tyee_batch *b, tyee_sim **sim) {
    if (!b || !sim) return fail(TYEE_EINVAL, "null argument");
    *sim = b->sim.get();
    return TYEE_OK;
}

int tyee_batch_set_state(tyee_batch *b, int64_t k, int32_t field, const double *host) {
    if (!member_ok(b, k) || !host) return fail(TYEE_EINVAL, "bad member or null array");
    tyee::Sim &s = b->sim->s;
    std::vector<double> v;
    if (field == TYEE_FIELD_E) {
        const int64_t o = b->off_e[k], n = b->off_e[k + 1] - o;
        v.resize(n);
        for (int64_t r = 0; r < n; ++r) {
            const int32_t i = s.perm_e[o + r];
            v[r] = (s.R[i] >= 0 && s.L[i] >= 0) ? s.scale(i) * host[i - o] : 0.0;
        }
        return tyee::upload_slice(s, s.Et(), o, v);
    }
    if (field == TYEE_FIELD_B) {
        const int64_t o = b->off_t[k], n = b->off_t[k + 1] - o;
        v.resize(n);
        for (int64_t r = 0; r < n; ++r) v[r] = host[s.perm_t[o + r] - o];
        return tyee::upload_slice(s, s.B(), o, v);
    }
    return fail(TYEE_EINVAL, "batches carry E and B only");
}

int tyee_batch_get_state(tyee_batch *b, int64_t k, int32_t field, double *host) {
    if (!member_ok(b, k) || !host) return fail(TYEE_EINVAL, "bad member or null array");
    tyee::Sim &s = b->sim->s;
    std::vector<double> v;
    int rc;
    if (field == TYEE_FIELD_E) {
        const int64_t o = b->off_e[k], n = b->off_e[k + 1] - o;
        if ((rc = tyee::download_slice(s, s.Et(), o, n, v))) return rc;
        for (int64_t r = 0; r < n; ++r) {
            const int32_t i = s.perm_e[o + r];
            host[i - o] = v[r] / s.scale(i);
        }
        return TYEE_OK;
    }
    if (field == TYEE_FIELD_B) {
        const int64_t o = b->off_t[k], n = b->off_t[k + 1] - o;
        if ((rc = tyee::download_slice(s, s.B(), o, n, v))) return rc;
        for (int64_t r = 0; r < n; ++r) host[s.perm_t[o + r] - o] = v[r];
        return TYEE_OK;
    }
    return fail(TYEE_EINVAL, "batches carry E and B only");
}

int tyee_batch_reorder(tyee_batch *b, int32_t kind, uint64_t seed) {
    if (!b) return fail(TYEE_EINVAL, "null batch");
    std::vector<double> E, B;
    int rc = save_fields(*b, E, B);
    if (rc) return rc;
    // canonical copies of the fields survive the renumbering
    tyee::Sim &s0 = b->sim->s;
    std::vector<double> Ec(s0.ne), Bc(s0.nt);
    for (int64_t k = 0; k < s0.ne; ++k) Ec[s0.perm_e[k]] = E[k];
    for (int64_t k = 0; k < s0.nt; ++k) Bc[s0.perm_t[k]] = B[k];
    const int64_t step = s0.step;
    for (auto &m : b->members)
        if ((rc = tyee::reorder_mesh(m, kind, seed))) return rc;
    if ((rc = rebuild(*b))) return rc;
    tyee::Sim &s = b->sim->s;
    for (int64_t k = 0; k < s.ne; ++k) E[k] = Ec[s.perm_e[k]];
    for (int64_t k = 0; k < s.nt; ++k) B[k] = Bc[s.perm_t[k]];
    s.step = step;
    rc = tyee::upload_slice(s, s.Et(), 0, E);
    return rc ? rc : tyee::upload_slice(s, s.B(), 0, B);
}

int tyee_batch_set_fusion(tyee_batch *b, int32_t k, int32_t tile) {
    if (!b) return fail(TYEE_EINVAL, "null batch");
    int rc = tyee_sim_set_fusion(b->sim.get(), k, tile);
    if (rc) return rc;
    b->fusion = b->sim->s.fusion;
    b->tile = tile;
    return TYEE_OK;
}

int tyee_batch_set_graph(tyee_batch *b, int32_t launches) {
    if (!b) return fail(TYEE_EINVAL, "null batch");
    int rc = tyee_sim_set_graph(b->sim.get(), launches);
    if (!rc) b->graph = launches;
    return rc;
}

int tyee_batch_step(tyee_batch *b, int64_t n) {
    if (!b) return fail(TYEE_EINVAL, "null batch");
    return tyee_sim_step(b->sim.get(), n);
}

int tyee_batch_sync(tyee_batch *b) {
    if (!b) return fail(TYEE_EINVAL, "null batch");
    return tyee_sim_sync(b->sim.get());
}

int tyee_batch_info(const tyee_batch *b, int64_t out[4]) {
    if (!b || !out) return fail(TYEE_EINVAL, "null argument");
    out[0] = int64_t(b->members.size());
    out[1] = b->merged.nt;
    out[2] = b->merged.ne;
    out[3] = b->merged.nv;
    return TYEE_OK;
}

int tyee_batch_tune(tyee_batch *b, int64_t steps_per_trial, tyee_tune_result *results, int64_t capacity,
                    int64_t *n_results) {
    return tyee_batch_tune_progress(b, steps_per_trial, results, capacity, n_results, nullptr, nullptr);
}

int tyee_batch_tune_progress(tyee_batch *b, int64_t steps_per_trial, tyee_tune_result *results,
                             int64_t capacity, int64_t *n_results, tyee_tune_progress on_trial, void *user) {
    if (!b || steps_per_trial <= 0 || (capacity > 0 && !results)) return fail(TYEE_EINVAL, "bad tune arguments");
    const int32_t orders[] = {TYEE_ORDER_MORTON, TYEE_ORDER_RCM};
    const int32_t depths[] = {1, 2, 4, 6, 8};
    const int32_t tiles[] = {1024, 1536, 2048, 3072};
    std::vector<tyee_tune_result> all;
    // canonical save of the fields and step count
    std::vector<double> E, B;
    int rc = save_fields(*b, E, B);
    if (rc) return rc;
    const int64_t step0 = b->sim->s.step;
    {
        tyee::Sim &s0 = b->sim->s;
        std::vector<double> Ec(s0.ne), Bc(s0.nt);
        for (int64_t k = 0; k < s0.ne; ++k) Ec[s0.perm_e[k]] = E[k];
        for (int64_t k = 0; k < s0.nt; ++k) Bc[s0.perm_t[k]] = B[k];
        E.swap(Ec);
        B.swap(Bc);
    }
    auto restore = [&](tyee_batch &bb) -> int {
        tyee::Sim &s = bb.sim->s;
        std::vector<double> e(s.ne), t(s.nt);
        for (int64_t k = 0; k < s.ne; ++k) e[k] = E[s.perm_e[k]];
        for (int64_t k = 0; k < s.nt; ++k) t[k] = B[s.perm_t[k]];
        s.step = step0;
        int r = tyee::upload_slice(s, s.Et(), 0, e);
        return r ? r : tyee::upload_slice(s, s.B(), 0, t);
    };
    tyee_tune_result best{};
    best.ms_per_step = INFINITY;
    for (int32_t order : orders) {
        for (auto &m : b->members)
            if ((rc = tyee::reorder_mesh(m, order, 0))) return rc;
        if ((rc = rebuild(*b)) || (rc = restore(*b))) return rc;
        for (int32_t K : depths) {
            for (int32_t tile : tiles) {
                if (K == 1 && tile != tiles[0]) continue;
                tyee_sim *sim = b->sim.get();
                if ((rc = tyee_sim_set_fusion(sim, K, K == 1 ? 0 : tile))) return rc;
                const int64_t span = int64_t(K) * std::max(1, b->graph);
                const int64_t n = std::max<int64_t>(span, (steps_per_trial + span - 1) / span * span);
                if ((rc = tyee_sim_step(sim, span))) return rc;  // warm-up (builds tiles, graph)
                if ((rc = tyee_sim_step(sim, n))) return rc;
                double ms = 0.0;
                if ((rc = tyee_sim_last_step_ms(sim, &ms))) return rc;
                // a depth whose tiles do not fit fell back to single steps: record what ran
                const int32_t ran = b->sim->s.fusion;
                tyee_tune_result r{order, ran, ran == 1 ? 0 : tile, ms / double(n)};
                all.push_back(r);
                if (on_trial) on_trial(&r, user);
                if (r.ms_per_step < best.ms_per_step) best = r;
                if ((rc = restore(*b))) return rc;
            }
        }
    }
    // apply the winner
    for (auto &m : b->members)
        if ((rc = tyee::reorder_mesh(m, best.order, 0))) return rc;
    b->fusion = best.steps_per_launch;
    b->tile = best.tile_tris;
    if ((rc = rebuild(*b)) || (rc = restore(*b))) return rc;
    for (int64_t r = 0; r < std::min<int64_t>(capacity, int64_t(all.size())); ++r) results[r] = all[r];
    if (n_results) *n_results = int64_t(all.size());
    return TYEE_OK;
}

void tyee_batch_destroy(tyee_batch *b) { delete b; }

}  // extern "C"
