// Simulation object shared by the runtime (sim.hip) and the fused tile kernels (fused.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "internal.hpp"
#include "tile.hpp"

#define TYEE_HIP(call)                                                                           \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return ::tyee::fail(TYEE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace tyee {

constexpr int kBlock = 256;
inline int blocks_for(int64_t n) { return int((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------------------
// simulation object
// ---------------------------------------------------------------------------------------

struct DeviceBuffer {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;  // false: caller memory bound with tyee_sim_bind_external
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer &) = delete;
    DeviceBuffer &operator=(const DeviceBuffer &) = delete;
    ~DeviceBuffer() {
        if (p && owned) (void)hipFree(p);
    }
    // (Re)allocate n bytes; an existing buffer of the same size is kept, so device
    // addresses captured in a graph stay valid across state uploads.
    int alloc(size_t n) {
        if (p && bytes == n) return TYEE_OK;
        if (!owned) return fail(TYEE_EINVAL, "a bound external buffer cannot be resized");
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = n;
        if (n == 0) return TYEE_OK;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(TYEE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        return TYEE_OK;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
    // Use caller memory of n bytes (not freed here); frees what this buffer owned.
    void borrow(void *ptr, size_t n) {
        if (p && owned) (void)hipFree(p);
        p = ptr;
        bytes = n;
        owned = false;
    }
    // Take ownership of memory allocated with hipMalloc (n bytes).
    void adopt(void *ptr, size_t n) {
        if (p && owned) (void)hipFree(p);
        p = ptr;
        bytes = n;
        owned = true;
    }
};

// Per-launch HIP-event timing of the stepping kernels (enabled per kernel kind).  A ring
// of event pairs keeps the queue deep: only the oldest pair is waited for when it fills.
struct LaunchTimer {
    static constexpr int kKinds = 6;
    static constexpr size_t kRing = 1024;
    struct Pair {
        int kind = 0;
        hipEvent_t start = nullptr, stop = nullptr;
    };
    uint32_t mask = 0;
    std::vector<Pair> ring;
    size_t head = 0, pending = 0;
    int64_t count[kKinds] = {0, 0, 0, 0, 0, 0};
    double total_ms[kKinds] = {0, 0, 0, 0, 0, 0};

    ~LaunchTimer() {
        for (auto &p : ring) {
            if (p.start) (void)hipEventDestroy(p.start);
            if (p.stop) (void)hipEventDestroy(p.stop);
        }
    }
    void reset(uint32_t m) {
        mask = m;
        std::fill(count, count + kKinds, 0);
        std::fill(total_ms, total_ms + kKinds, 0.0);
    }
    int retire_oldest() {
        Pair &p = ring[(head + ring.size() - pending) % ring.size()];
        TYEE_HIP(hipEventSynchronize(p.stop));
        float ms = 0.0f;
        TYEE_HIP(hipEventElapsedTime(&ms, p.start, p.stop));
        count[p.kind] += 1;
        total_ms[p.kind] += ms;
        --pending;
        return TYEE_OK;
    }
    int drain() {
        while (pending > 0) {
            int rc = retire_oldest();
            if (rc) return rc;
        }
        return TYEE_OK;
    }
    // returns the ring slot used, or -1 when this kind is not timed
    int begin(int kind, hipStream_t s, int *rc) {
        *rc = TYEE_OK;
        if (!(mask & (1u << kind))) return -1;
        if (ring.empty()) ring.resize(kRing);
        if (pending == ring.size() && (*rc = retire_oldest())) return -1;
        Pair &p = ring[head];
        if (!p.start && (hipEventCreate(&p.start) != hipSuccess || hipEventCreate(&p.stop) != hipSuccess)) {
            *rc = fail(TYEE_EDEVICE, "hipEventCreate failed");
            return -1;
        }
        p.kind = kind;
        if (hipEventRecord(p.start, s) != hipSuccess) {
            *rc = fail(TYEE_EDEVICE, "hipEventRecord failed");
            return -1;
        }
        int slot = int(head);
        head = (head + 1) % ring.size();
        ++pending;
        return slot;
    }
    int end(int slot, hipStream_t s) {
        if (slot < 0) return TYEE_OK;
        TYEE_HIP(hipEventRecord(ring[slot].stop, s));
        return TYEE_OK;
    }
};

struct Tiling;


// Soft-source waveform g(t) = sin(omega t) sin^2(pi t / T) for 0 <= t < T, T = cycles 2 pi/omega.
inline double waveform(double t, double omega, double cycles) {
    const double T = cycles * 2.0 * M_PI / omega;
    if (!(t >= 0.0 && t < T)) return 0.0;
    const double s = std::sin(M_PI * t / T);
    return std::sin(omega * t) * s * s;
}

struct Probe {
    int32_t field = 0;
    int64_t n = 0, every = 1, capacity = 0, taken = 0;
    std::vector<int32_t> ids;     // canonical ids
    DeviceBuffer slots;           // device slots (special-list index for J)
    DeviceBuffer samples;         // [capacity][n] raw device values
};

struct Sim {
    bool f64 = false;
    size_t esz = 4;
    double dt = 0.0;                           // time step (of the first mesh in a batch)
    std::vector<double> dt_tri, dt_edge;       // per canonical cell (batches mix meshes)
    hipStream_t stream = nullptr;
    bool own_stream = false;                   // created by the library (caller passed NULL)
    int device = 0;                            // HIP device current at creation
    int graph_launches = 0;                    // fused launches per captured graph (0 = eager)
    hipGraphExec_t graph = nullptr;
    bool graph_dirty = true;
    int graph_K = 0, graph_cur = -1;
    int64_t nv = 0, ne = 0, nt = 0;
    int64_t step = 0;
    int fusion = 1;
    int tile_tris = 0;                         // 0 = default tile size for the fusion depth
    int cur = 0;                               // which of the two field buffers is current
    std::vector<double> ce_dev, nb_dev;        // half-step coefficients in device numbering
    std::unique_ptr<struct Tiling> tiling;

    // host copies (canonical numbering)
    std::vector<int32_t> perm_t, perm_e, slot_t, slot_e;
    std::vector<int32_t> edge, R, L, A;
    std::vector<int8_t> sgn;
    std::vector<double> elen, d, hR, hL, S;
    std::vector<uint8_t> node_outer;
    std::vector<double> gamma;  // per canonical edge
    std::vector<double> wp2_edge;
    double nu = 0.0;
    std::vector<int32_t> src_edge;
    std::vector<double> src_w;
    double src_omega = 1.0, src_cycles = 1.0;

    // device arrays, device numbering
    DeviceBuffer Et_buf[2], B_buf[2], cE, nB, RL, A0, A1, A2;
    DeviceBuffer &Et() { return Et_buf[cur]; }
    DeviceBuffer &B() { return B_buf[cur]; }
    // special edges (plasma and/or source)
    int64_t n_special = 0;
    std::vector<int32_t> sp_edge;  // canonical edge of each special entry
    std::vector<uint8_t> sp_plasma;
    DeviceBuffer sp_slot, sp_j_buf[2], sp_ca, sp_cb, sp_w;
    DeviceBuffer sp_delta;         // [steps of one launch][n_special] decrements, for the charge
    DeviceBuffer &sp_j() { return sp_j_buf[cur]; }  // current flips with the field buffers
    // nodal charge
    int64_t n_qnode = 0;
    DeviceBuffer Q, q_node, q_off, q_inc, q_coef;

    // diagnostics tables (FP64 weights in device numbering), built on first use
    bool diag_ready = false;
    DeviceBuffer diag_wE, diag_inv_scale, diag_S, diag_dtS, diag_partial;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    LaunchTimer timer;
    std::vector<std::unique_ptr<Probe>> probes;

    ~Sim();

    double scale(int64_t i) const { return gamma[i] * elen[i]; }  // Et = scale * E
    // Per-launch timing of kernels that a graph would hold bypasses graph replay, unless
    // whole replays are timed too: then replays stay on and the other kinds time only the
    // launches made outside a graph (a remainder shorter than one graph span).
    bool timer_wants_kernels() const {
        const uint32_t g = 1u << TYEE_KERNEL_GRAPH;
        return (timer.mask & ~g) != 0 && (timer.mask & g) == 0;
    }
};


// Temporal tiling for the fused K-step kernel (built by fused.hip); TileInfo is in tile.hpp.
struct Tiling {
    int K = 0, tile = 0, threads = 0, rt = 0, re = 0;
    int64_t ntiles = 0, maxT = 0, maxE = 0, sumT = 0, sumE = 0;
    DeviceBuffer info, tl_glob, tl_coef, tl_i0, tl_i1, el_glob, el_coef, el_idx;
    DeviceBuffer el_sp;     // special-list index of each local edge, -1 if none (when specials exist)
    DeviceBuffer tile_ids;  // plain-class tiles, then tiles holding a special edge
    int64_t n_sp_tiles = 0;
    bool has_sp = false;
    std::vector<int32_t> h_tl_glob, h_el_glob;  // local cell -> device slot (for coefficient refresh)
};

int build_tiling(Sim &s, int K, int tile_tris);
int init_sim(Sim &s, const Mesh &m, int32_t prec, const std::vector<double> &dt_tri,
             const std::vector<double> &dt_edge, void *stream);
int refresh_tiling_coefficients(Sim &s);
template <typename T> int launch_fused(Sim &s, int k);

}  // namespace tyee

struct tyee_sim {
    tyee::Sim s;
};
