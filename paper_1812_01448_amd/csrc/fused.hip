// Temporally fused leap-frog: K steps of the edge and triangle half-steps (eqs. 3-4 of
// arXiv:1812.01448) in one launch, one work-group per tile of the device numbering.
//
// Locality is what makes the scheme cheap to fuse: one step moves information by one
// triangle.  A tile owns a run of consecutive device triangles (the core).  Its work-group
// also loads K rings of neighbouring triangles (level m = ring distance from the core) and
// every edge of the levels below K.  In step s = 1..K it advances the edges and triangles
// of level <= K - s; after K steps the core triangles and the edges it owns (an edge belongs
// to the tile of its lower-numbered triangle) are exact and are written out.  Everything
// between the first load and the final store stays on chip:
//   - field values in LDS (they are exchanged between work-items each half-step),
//   - coefficients and local neighbour indices in VGPRs (each work-item keeps its cells),
// so HBM sees one read of the tile's cells and one write of its own cells per K steps.
// Core triangles are a run of device slots, and so are the owned edges under the Morton and
// RCM numberings (edges numbered by first appearance over the triangles): their slots are
// computed, only halo cells carry a stored slot.
// Work-groups read the "in" buffers and write the "out" buffers, so a tile never sees a
// neighbour's already-advanced values; the runtime swaps the two buffers after each launch.
// The per-cell arithmetic is exactly that of k_edge / k_tri (same fma, same q order), so any
// fusion depth gives bit-identical fields.
//
// Special edges (plasma current, eq. 5, and the soft source) ride along: the work-item that
// holds such an edge also holds its current j and Drude coefficients and applies the same
// correction k_special does, in the same order, just before the edge half-step.  Halo copies
// of j advance redundantly like the fields; each tile writes back j of its own edges (into
// the other j buffer) and, per step, their decrements, from which k_charge then advances the
// nodal charge step by step, so E, B, j and Q stay bit-identical to single-step launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>

#include "kernels.hpp"
#include "sim.hpp"

namespace tyee {

namespace {

constexpr int kFusedThreads = 1024;

template <typename T> __device__ __forceinline__ T lds_signed(const T *v, uint32_t half);
template <> __device__ __forceinline__ float lds_signed<float>(const float *v, uint32_t half) {
    const float x = v[half & 0x7FFFu];
    return __uint_as_float(__float_as_uint(x) ^ ((half & 0x8000u) << 16));
}
template <> __device__ __forceinline__ double lds_signed<double>(const double *v, uint32_t half) {
    const double x = v[half & 0x7FFFu];
    return __longlong_as_double(__double_as_longlong(x) ^ (static_cast<long long>(half & 0x8000u) << 48));
}

// Arguments of the special-edge variant (unused by the plain kernel).
template <typename T> struct SpecialArgs {
    const int32_t *el_sp;  // per local edge: special-list index or -1
    const T *j_in;
    T *j_out;
    const T *ca, *cb, *w;  // Drude coefficients and source weight per special entry
    T *delta;              // [step][nsp] decrements of owned special edges
    int nsp;
    T dt;
    T g[kMaxFusion];       // source waveform at the midpoint of each step of the launch
};

template <typename T, int NT, int RT, int RE, bool SP>
__global__ __launch_bounds__(NT) void k_fused(int K, int lds_tris, const TileInfo *__restrict__ tiles,
                                              const T *__restrict__ Et_in, const T *__restrict__ B_in,
                                              T *__restrict__ Et_out, T *__restrict__ B_out,
                                              const int32_t *__restrict__ tl_glob, const T *__restrict__ tl_coef,
                                              const uint32_t *__restrict__ tl_i0, const uint16_t *__restrict__ tl_i1,
                                              const int32_t *__restrict__ el_glob, const T *__restrict__ el_coef,
                                              const uint32_t *__restrict__ el_idx,
                                              const int32_t *__restrict__ tile_ids, const SpecialArgs<T> sp) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *sB = reinterpret_cast<T *>(lds_raw);
    T *sE = sB + lds_tris;
    int t = xcd_group(blockIdx.x, gridDim.x);
    if (tile_ids) t = tile_ids[t];  // a subset of the tiles (one class of a split launch)
    const TileInfo &ti = tiles[t];
    const int tid = threadIdx.x;
    const int nT = ti.cntT[K], nE = ti.cntE[K - 1];

    T vb[RT], cb[RT], ve[RE], ce[RE];
    uint32_t i0[RT], i1[RT], ie[RE];
    int32_t gt[RT], ge[RE];
    int spk[RE];
    T jr[RE], sa[RE], sb[RE], sw[RE];
    // The loads are issued in three waves so that a work-item keeps all of them in flight at
    // once: the stored slots of halo cells, then the coefficient and index tables, then the
    // field values through the slots.  Loading cell by cell, with the slot chosen at the load,
    // serialises every cell on two memory round trips.  Table and value loads are unconditional
    // (cells past the tile read the tile's last table entry and slot 0, and are never used),
    // so no branch sits between them and the compiler waits once.
    const bool own_run = ti.own_base >= 0;
    // The waves of a tile being loaded run at a raised priority until its cells are staged, so
    // on a CU whose other work-group is in its LDS steps the loads are issued first and their
    // latency overlaps those steps (measured: 10.84 -> 10.66 us per step at 4 steps per launch).
    __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int l = tid + r * NT;
        gt[r] = l < ti.n_core ? ti.core_base + l : 0;
        if (l >= ti.n_core && l < nT) gt[r] = tl_glob[ti.tri_off + l];
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int l = tid + r * NT;
        ge[r] = (own_run && l < ti.n_own) ? ti.own_base + l : 0;
        if ((!own_run || l >= ti.n_own) && l < nE) ge[r] = el_glob[ti.edge_off + l];
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int p = ti.tri_off + min(tid + r * NT, nT - 1);
        cb[r] = tl_coef[p];
        i0[r] = tl_i0[p];
        i1[r] = tl_i1[p];
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int l = tid + r * NT;
        const int p = ti.edge_off + min(l, nE - 1);
        ce[r] = el_coef[p];
        ie[r] = el_idx[p];
        spk[r] = -1;
        jr[r] = sa[r] = sb[r] = sw[r] = T(0);
        if constexpr (SP) spk[r] = l < nE ? sp.el_sp[p] : -1;
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) vb[r] = B_in[gt[r]];
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        ve[r] = Et_in[ge[r]];
        if constexpr (SP) {
            if (spk[r] >= 0) {
                jr[r] = sp.j_in[spk[r]];
                sa[r] = sp.ca[spk[r]];
                sb[r] = sp.cb[spk[r]];
                sw[r] = sp.w[spk[r]];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int l = tid + r * NT;
        if (l < nT) sB[l] = vb[r];
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int l = tid + r * NT;
        if (l < nE) sE[l] = ve[r];
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();

    for (int s = 1; s <= K; ++s) {
        const int le = ti.cntE[K - s], lt = ti.cntT[K - s];
#pragma unroll
        for (int r = 0; r < RE; ++r) {
            const int l = tid + r * NT;
            if (l < le) {
                const T diff = sB[ie[r] & 0xFFFFu] - sB[ie[r] >> 16];
                T e = ve[r];
                if constexpr (SP) {
                    if (spk[r] >= 0) {  // k_special's correction, same operations
                        const T j = fma(sa[r], jr[r], sb[r] * e);
                        jr[r] = j;
                        const T dl = fma(sp.dt, j, sw[r] * sp.g[s - 1]);
                        if (l < ti.n_own) sp.delta[int64_t(s - 1) * sp.nsp + spk[r]] = dl;
                        e = e - dl;
                    }
                }
                ve[r] = fma(ce[r], diff, e);
                sE[l] = ve[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            const int l = tid + r * NT;
            if (l < lt) {
                const T circ = (lds_signed(sE, i0[r] & 0xFFFFu) + lds_signed(sE, i0[r] >> 16)) +
                               lds_signed(sE, i1[r]);
                vb[r] = fma(cb[r], circ, vb[r]);
                sB[l] = vb[r];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int l = tid + r * NT;
        if (l < ti.n_core) B_out[ti.core_base + l] = vb[r];
    }
#pragma unroll
    for (int r = 0; r < RE; ++r) {
        const int l = tid + r * NT;
        if (l < ti.n_own) {
            Et_out[ge[r]] = ve[r];
            if constexpr (SP) {
                if (spk[r] >= 0) sp.j_out[spk[r]] = jr[r];
            }
        }
    }
}

// Register capacities (cells per work-item) compiled for the fused kernel.
struct Capacity {
    int rt, re;
};
constexpr Capacity kMenu[] = {{2, 3}, {3, 4}, {3, 5}, {4, 6}, {5, 7}, {6, 9}, {7, 10}, {8, 12}};

// Tiles without any special edge (the plain class, listed first) run the plain kernel; the
// few that hold one run the special variant, whose extra registers would otherwise lower the
// occupancy of every tile.  Both read the "in" buffers and write disjoint cells of the "out"
// buffers.  The charge update of the K steps follows; it reads only the decrements the
// special-class tiles wrote.
template <typename T, int RT, int RE>
int launch_one(Sim &s, int K, const T *ei, const T *bi, T *eo, T *bo, const SpecialArgs<T> &sp) {
    Tiling &tg = *s.tiling;
    const size_t lds = size_t(tg.maxT + tg.maxE) * sizeof(T);
    const int64_t n_plain = tg.ntiles - tg.n_sp_tiles;
    const int32_t *ids = tg.n_sp_tiles > 0 ? tg.tile_ids.as<int32_t>() : nullptr;
    if (n_plain > 0)
        k_fused<T, kFusedThreads, RT, RE, false><<<int(n_plain), kFusedThreads, lds, s.stream>>>(
            K, int(tg.maxT), tg.info.as<TileInfo>(), ei, bi, eo, bo, tg.tl_glob.as<int32_t>(), tg.tl_coef.as<T>(),
            tg.tl_i0.as<uint32_t>(), tg.tl_i1.as<uint16_t>(), tg.el_glob.as<int32_t>(), tg.el_coef.as<T>(),
            tg.el_idx.as<uint32_t>(), ids, SpecialArgs<T>{});
    if (tg.n_sp_tiles > 0) {
        k_fused<T, kFusedThreads, RT, RE, true><<<int(tg.n_sp_tiles), kFusedThreads, lds, s.stream>>>(
            K, int(tg.maxT), tg.info.as<TileInfo>(), ei, bi, eo, bo, tg.tl_glob.as<int32_t>(), tg.tl_coef.as<T>(),
            tg.tl_i0.as<uint32_t>(), tg.tl_i1.as<uint16_t>(), tg.el_glob.as<int32_t>(), tg.el_coef.as<T>(),
            tg.el_idx.as<uint32_t>(), ids + n_plain, sp);
        launch_charge<T>(s.stream, s.n_qnode, s.q_node.as<int32_t>(), s.q_off.as<int32_t>(), s.q_inc.as<int32_t>(),
                         s.q_coef.as<T>(), s.sp_delta.as<T>(), K, int(s.n_special), s.Q.as<T>());
    }
    return TYEE_OK;
}

template <typename T> int upload_vec(Sim &s, DeviceBuffer &buf, const std::vector<T> &v) {
    int rc = buf.alloc(v.size() * sizeof(T));
    if (rc || v.empty()) return rc;
    TYEE_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s.stream));
    TYEE_HIP(hipStreamSynchronize(s.stream));
    return TYEE_OK;
}

// Default tile size for a fusion depth: the largest tile whose K halo rings still fit the
// register capacity that lets two 1024-item work-groups share a CU (torus1415 FP32 sweep).
int default_tile(bool f64, int K) {
    if (f64) return K >= 4 ? 1024 : 2048;
    if (K >= 8) return 1024;
    if (K >= 6) return 1536;
    return K == 5 ? 1792 : 2048;
}

}  // namespace

int refresh_tiling_coefficients(Sim &s) {
    Tiling &tg = *s.tiling;
    std::vector<double> tc(tg.h_tl_glob.size()), ec(tg.h_el_glob.size());
    for (size_t p = 0; p < tc.size(); ++p) tc[p] = s.nb_dev[tg.h_tl_glob[p]];
    for (size_t p = 0; p < ec.size(); ++p) ec[p] = s.ce_dev[tg.h_el_glob[p]];
    if (s.f64) {
        int rc = upload_vec(s, tg.tl_coef, tc);
        return rc ? rc : upload_vec(s, tg.el_coef, ec);
    }
    std::vector<float> tf(tc.begin(), tc.end()), ef(ec.begin(), ec.end());
    int rc = upload_vec(s, tg.tl_coef, tf);
    return rc ? rc : upload_vec(s, tg.el_coef, ef);
}

// Cut the device numbering into tiles of `tile` consecutive triangles and record, for each,
// its K rings of neighbours and the edges they need (see the file comment).
int build_tiling(Sim &s, int K, int tile_tris) {
    if (K < 2 || K > kMaxFusion) return fail(TYEE_EINVAL, "fusion depth must be 2..8");
    int device = 0, lds_limit = 65536;
    TYEE_HIP(hipGetDevice(&device));
    TYEE_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
    const int64_t nt = s.nt, ne = s.ne;
    const size_t esz = s.f64 ? 8 : 4;

    // device-slot adjacency: neighbour triangle, edge slot and sign of each side
    std::vector<int32_t> nbr(3 * nt), eslot(3 * nt);
    std::vector<int8_t> esgn(3 * nt);
    for (int64_t k = 0; k < nt; ++k) {
        const int32_t j = s.perm_t[k];
        for (int q = 0; q < 3; ++q) {
            const int32_t i = s.A[3 * j + q];
            const bool inner = s.R[i] >= 0 && s.L[i] >= 0;
            nbr[3 * k + q] = inner ? s.slot_t[s.R[i] == j ? s.L[i] : s.R[i]] : -1;
            eslot[3 * k + q] = s.slot_e[i];
            esgn[3 * k + q] = s.sgn[3 * j + q];
        }
    }
    std::vector<int32_t> eR(ne), eL(ne);  // triangle slots either side of each edge slot
    for (int64_t m = 0; m < ne; ++m) {
        const int32_t i = s.perm_e[m];
        const int32_t r = s.R[i] >= 0 ? s.slot_t[s.R[i]] : -1, l = s.L[i] >= 0 ? s.slot_t[s.L[i]] : -1;
        eR[m] = r >= 0 ? r : l;
        eL[m] = l >= 0 ? l : r;
    }

    int tile = tile_tris > 0 ? tile_tris : default_tile(s.f64, K);
    for (;;) {
        auto tg = std::make_unique<Tiling>();
        tg->K = K;
        tg->tile = tile;
        tg->threads = kFusedThreads;
        tg->ntiles = (nt + tile - 1) / tile;
        std::vector<TileInfo> info(tg->ntiles);
        std::vector<int32_t> level(nt, -1), local_t(nt, -1), local_e(ne, -1);
        std::vector<uint32_t> ti0, eidx;
        std::vector<uint16_t> ti1;
        bool too_big = false;
        for (int64_t t = 0; t < tg->ntiles && !too_big; ++t) {
            const int32_t c0 = int32_t(t * tile), c1 = int32_t(std::min<int64_t>(nt, (t + 1) * tile));
            std::vector<int32_t> tris;
            std::vector<int32_t> cnt_t(K + 1, 0);
            for (int32_t k = c0; k < c1; ++k) {
                level[k] = 0;
                tris.push_back(k);
            }
            cnt_t[0] = int32_t(tris.size());
            size_t ring_begin = 0;
            for (int r = 1; r <= K; ++r) {
                const size_t ring_end = tris.size();
                for (size_t a = ring_begin; a < ring_end; ++a)
                    for (int q = 0; q < 3; ++q) {
                        const int32_t o = nbr[3 * tris[a] + q];
                        if (o >= 0 && level[o] < 0) {
                            level[o] = r;
                            tris.push_back(o);
                        }
                    }
                std::sort(tris.begin() + ring_end, tris.end());
                ring_begin = ring_end;
                cnt_t[r] = int32_t(tris.size());
            }
            for (size_t a = 0; a < tris.size(); ++a) local_t[tris[a]] = int32_t(a);

            // edges of levels 0..K-1: owned first (by slot), then by (level, slot)
            std::vector<std::pair<int64_t, int32_t>> edges;  // (sort key, edge slot)
            for (int32_t a = 0; a < cnt_t[K - 1]; ++a)
                for (int q = 0; q < 3; ++q) {
                    const int32_t m = eslot[3 * tris[a] + q];
                    if (local_e[m] >= 0) continue;
                    local_e[m] = 0;
                    const int32_t lev = std::min(level[eR[m]], level[eL[m]]);
                    const int32_t owner = std::min(eR[m], eL[m]);
                    const bool own = owner >= c0 && owner < c1;
                    const int64_t key = own ? -1 : lev;
                    edges.push_back({key * (int64_t(ne) + 1) + m, m});
                }
            std::sort(edges.begin(), edges.end());
            std::vector<int32_t> cnt_e(K + 1, 0);
            int32_t n_own = 0;
            for (size_t a = 0; a < edges.size(); ++a) {
                const int32_t m = edges[a].second;
                local_e[m] = int32_t(a);
                const int32_t owner = std::min(eR[m], eL[m]);
                if (owner >= c0 && owner < c1) ++n_own;
                const int32_t lev = std::min(level[eR[m]], level[eL[m]]);
                for (int v = lev; v <= K; ++v) ++cnt_e[v];
            }
            if (tris.size() > 32767 || edges.size() > 32767) too_big = true;

            TileInfo &ti = info[t];
            ti.n_core = c1 - c0;
            ti.n_own = n_own;
            ti.core_base = c0;
            ti.own_base = n_own > 0 ? edges[0].second : -1;
            for (int32_t a = 0; a < n_own && ti.own_base >= 0; ++a)
                if (edges[a].second != ti.own_base + a) ti.own_base = -1;  // not a run: stored slots
            ti.tri_off = int32_t(tg->h_tl_glob.size());
            ti.edge_off = int32_t(tg->h_el_glob.size());
            for (int v = 0; v <= 8; ++v) {
                ti.cntT[v] = cnt_t[std::min(v, K)];
                ti.cntE[v] = cnt_e[std::min(v, K)];
            }
            for (size_t a = 0; a < tris.size(); ++a) {
                const int32_t k = tris[a];
                tg->h_tl_glob.push_back(k);
                uint32_t h[3] = {0, 0, 0};
                if (level[k] < K)
                    for (int q = 0; q < 3; ++q)
                        h[q] = uint32_t(local_e[eslot[3 * k + q]]) | (esgn[3 * k + q] < 0 ? 0x8000u : 0u);
                ti0.push_back(h[0] | (h[1] << 16));
                ti1.push_back(uint16_t(h[2]));
            }
            for (auto &e : edges) {
                const int32_t m = e.second;
                tg->h_el_glob.push_back(m);
                eidx.push_back(uint32_t(local_t[eR[m]]) | (uint32_t(local_t[eL[m]]) << 16));
            }
            tg->maxT = std::max<int64_t>(tg->maxT, int64_t(tris.size()));
            tg->maxE = std::max<int64_t>(tg->maxE, int64_t(edges.size()));
            for (int32_t k : tris) level[k] = local_t[k] = -1;
            for (auto &e : edges) local_e[e.second] = -1;
        }
        const size_t lds = size_t(tg->maxT + tg->maxE) * esz;
        if (too_big || lds > size_t(lds_limit)) {
            if (tile_tris > 0 || tile <= 256)
                return fail(TYEE_EINVAL, "tiles do not fit the fused kernel at this depth");
            tile /= 2;
            continue;
        }
        // smallest compiled register capacity that holds every tile
        int pick = -1;
        for (int c = 0; c < int(sizeof(kMenu) / sizeof(kMenu[0])); ++c)
            if (int64_t(kMenu[c].rt) * kFusedThreads >= tg->maxT && int64_t(kMenu[c].re) * kFusedThreads >= tg->maxE) {
                pick = c;
                break;
            }
        if (pick < 0) {
            if (tile_tris > 0 || tile <= 256) return fail(TYEE_EINVAL, "tiles exceed the fused kernel capacity");
            tile /= 2;
            continue;
        }
        tg->rt = kMenu[pick].rt;
        tg->re = kMenu[pick].re;
        tg->sumT = int64_t(tg->h_tl_glob.size());
        tg->sumE = int64_t(tg->h_el_glob.size());
        // host-side bounds check of everything the kernel will index
        for (int32_t k : tg->h_tl_glob)
            if (k < 0 || k >= nt) return fail(TYEE_EINVAL, "internal: tile triangle slot out of range");
        for (int32_t m : tg->h_el_glob)
            if (m < 0 || m >= ne) return fail(TYEE_EINVAL, "internal: tile edge slot out of range");
        for (int64_t t = 0; t < tg->ntiles; ++t) {
            const TileInfo &ti = info[t];
            const int32_t nT = ti.cntT[K], nE = ti.cntE[K - 1];
            for (int32_t a = 0; a < nT; ++a) {
                const uint32_t w0 = ti0[ti.tri_off + a], w1 = ti1[ti.tri_off + a];
                if (a < ti.n_core && tg->h_tl_glob[ti.tri_off + a] != ti.core_base + a)
                    return fail(TYEE_EINVAL, "internal: core triangles are not a run of slots");
                if ((w0 & 0x7FFFu) >= uint32_t(nE) || ((w0 >> 16) & 0x7FFFu) >= uint32_t(nE) ||
                    (w1 & 0x7FFFu) >= uint32_t(nE))
                    return fail(TYEE_EINVAL, "internal: local edge index out of range");
            }
            for (int32_t a = 0; a < nE; ++a) {
                const uint32_t w = eidx[ti.edge_off + a];
                if (a < ti.n_own && ti.own_base >= 0 && tg->h_el_glob[ti.edge_off + a] != ti.own_base + a)
                    return fail(TYEE_EINVAL, "internal: owned edges are not a run of slots");
                if ((w & 0xFFFFu) >= uint32_t(nT) || (w >> 16) >= uint32_t(nT))
                    return fail(TYEE_EINVAL, "internal: local triangle index out of range");
            }
            if (ti.n_core > nT || ti.n_own > ti.cntE[0] || nT > tg->maxT || nE > tg->maxE)
                return fail(TYEE_EINVAL, "internal: tile counts out of range");
            for (int v = 1; v <= K; ++v)
                if (ti.cntT[v] < ti.cntT[v - 1] || ti.cntE[v] < ti.cntE[v - 1])
                    return fail(TYEE_EINVAL, "internal: tile levels not nested");
        }
        std::vector<int32_t> el_sp, ids;
        if (s.n_special > 0) {
            std::vector<int32_t> sp_of_slot(ne, -1);
            for (int64_t k = 0; k < s.n_special; ++k) sp_of_slot[s.slot_e[s.sp_edge[k]]] = int32_t(k);
            el_sp.resize(tg->h_el_glob.size());
            for (size_t p = 0; p < el_sp.size(); ++p) el_sp[p] = sp_of_slot[tg->h_el_glob[p]];
            tg->has_sp = true;
            // tile classes: no special edge among a tile's local edges -> plain kernel
            std::vector<int32_t> special_tiles;
            for (int64_t t = 0; t < tg->ntiles; ++t) {
                const TileInfo &ti = info[t];
                bool any = false;
                for (int32_t a = 0; a < ti.cntE[K - 1] && !any; ++a) any = el_sp[ti.edge_off + a] >= 0;
                (any ? special_tiles : ids).push_back(int32_t(t));
            }
            tg->n_sp_tiles = int64_t(special_tiles.size());
            ids.insert(ids.end(), special_tiles.begin(), special_tiles.end());
            for (int32_t v : el_sp)
                if (v >= int64_t(s.n_special)) return fail(TYEE_EINVAL, "internal: special index out of range");
        }
        int rc = upload_vec(s, tg->info, info);
        if (!rc && tg->has_sp) rc = upload_vec(s, tg->el_sp, el_sp);
        if (!rc && tg->has_sp) rc = upload_vec(s, tg->tile_ids, ids);
        if (!rc) rc = upload_vec(s, tg->tl_glob, tg->h_tl_glob);
        if (!rc) rc = upload_vec(s, tg->tl_i0, ti0);
        if (!rc) rc = upload_vec(s, tg->tl_i1, ti1);
        if (!rc) rc = upload_vec(s, tg->el_glob, tg->h_el_glob);
        if (!rc) rc = upload_vec(s, tg->el_idx, eidx);
        if (rc) return rc;
        s.tiling = std::move(tg);
        s.graph_dirty = true;
        return refresh_tiling_coefficients(s);
    }
}

template <typename T> int launch_fused(Sim &s, int k) {
    Tiling &tg = *s.tiling;
    if (k != tg.K || k < 2 || k > kMaxFusion) return fail(TYEE_EINVAL, "internal: fused depth mismatch");
    if (tg.has_sp != (s.n_special > 0)) return fail(TYEE_EINVAL, "internal: tiling out of date with specials");
    const T *ei = s.Et_buf[s.cur].as<T>(), *bi = s.B_buf[s.cur].as<T>();
    T *eo = s.Et_buf[1 - s.cur].as<T>(), *bo = s.B_buf[1 - s.cur].as<T>();
    SpecialArgs<T> sp{};
    if (tg.has_sp) {
        sp.el_sp = tg.el_sp.as<int32_t>();
        sp.j_in = s.sp_j_buf[s.cur].as<T>();
        sp.j_out = s.sp_j_buf[1 - s.cur].as<T>();
        sp.ca = s.sp_ca.as<T>();
        sp.cb = s.sp_cb.as<T>();
        sp.w = s.sp_w.as<T>();
        sp.delta = s.sp_delta.as<T>();
        sp.nsp = int(s.n_special);
        sp.dt = T(s.dt);
        for (int q = 0; q < k; ++q)
            sp.g[q] = T(waveform((double(s.step + q) + 0.5) * s.dt, s.src_omega, s.src_cycles));
    }
    int rc;
    switch (tg.rt * 100 + tg.re) {
    case 203: rc = launch_one<T, 2, 3>(s, k, ei, bi, eo, bo, sp); break;
    case 304: rc = launch_one<T, 3, 4>(s, k, ei, bi, eo, bo, sp); break;
    case 305: rc = launch_one<T, 3, 5>(s, k, ei, bi, eo, bo, sp); break;
    case 406: rc = launch_one<T, 4, 6>(s, k, ei, bi, eo, bo, sp); break;
    case 507: rc = launch_one<T, 5, 7>(s, k, ei, bi, eo, bo, sp); break;
    case 609: rc = launch_one<T, 6, 9>(s, k, ei, bi, eo, bo, sp); break;
    case 710: rc = launch_one<T, 7, 10>(s, k, ei, bi, eo, bo, sp); break;
    case 812: rc = launch_one<T, 8, 12>(s, k, ei, bi, eo, bo, sp); break;
    default: return fail(TYEE_EINVAL, "internal: no fused kernel for this capacity");
    }
    if (rc) return rc;
    s.cur = 1 - s.cur;
    return TYEE_OK;
}

template int launch_fused<float>(Sim &, int);
template int launch_fused<double>(Sim &, int);

}  // namespace tyee
