// Learned per-edge coefficient scale for the triangular Yee-like scheme, trained and applied
// on the GPU.
//
// Model: gamma_i = 1 + 0.1 tanh(w3 . tanh(W2 tanh(W1 x_i + b1) + b2) + b3) with
// x_i = (f_i - mu)/sd the normalised eight geometry features of edge i (8 -> 32 -> 32 -> 1,
// 1,377 parameters in the order W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3).  Scaling
// the eq. 3 and eq. 4 coefficients of an edge by the same gamma keeps metric (7) conserved.
//
// Training signal: the phase error that leap-frog itself produces on plane waves over small
// periodic training meshes.  Eliminating E from the two half-steps, x_n = B^{n+1/2} obeys
//   x_{n+1} = (2 - dt^2 K_gamma) x_n - x_{n-1},   (K_gamma x)_j = (1/S_j) sum_q gamma^2 |e|/d (x_j - x_nb),
// started from the exact wave exp(i(k.O -+ |k| dt/2)).  After N steps (about 2 radians of
// phase) the overlap z_N = sum_j S_j conj(exp(i k.O_j)) x_N,j gives eps = -arg(z_N/z_0)/(|k| N dt) - 1,
// and the loss is the mean of eps^2 over meshes and waves.  Its exact gradient pairs the
// forward sequence x_n with the second-kind Chebyshev sequence v_m (v_{-1} = 0, v_0 =
// exp(i k.O)) run backwards from m = N - 1 (the recurrence is reversible):
//   dz_N/dgamma_i = -2 dt^2 gamma_i (|e_i|/d_i) sum_n conj(v_{N-1-n,R} - v_{N-1-n,L}) (x_{n,R} - x_{n,L}).
// Both recurrences run in the difference form y_{n+1} = y_n - dt^2 K x_n, x_{n+1} = x_n + y_{n+1},
// which keeps the small per-step increments accurate in FP32.
//
// Kernels:
//   k_mlp_gamma     one work-item per edge: the MLP forward pass;
//   k_ts_adjoint    one work-group per (training mesh, wave): the whole mesh lives in LDS
//                   (up to 4096 triangles), each work-item keeps its triangles' state and its
//                   edges' accumulators in registers; forward pass, then the reversed pass
//                   with the per-edge accumulation; writes eps and the wave's share of dL/dgamma;
//                   work-groups are dispatched longest recurrence first, so the last ones to
//                   start are short and the launch ends with little idle time;
//   k_wave_sum      per edge: dL/dgamma summed over the waves in wave order;
//   k_stiff_reg     per stiff edge (d/|e| below a threshold): the pull of gamma toward its
//                   target, added to dL/dgamma (it lowers omega_max, so the eq. 20 step grows);
//   k_loss          one block: the loss from the eps values;
//   k_mlp_backward  per block: forward + backward of its edges, the per-edge activation and
//                   delta vectors staged in LDS, then each work-item accumulates the gradient
//                   of its own parameters over the staged edges (no atomics);
//   k_grad_reduce   per parameter: sum of the block partials in block order;
//   k_adam          per parameter: Adam update.
// Every reduction has a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <memory>

#include "internal.hpp"
#include "sim.hpp"

namespace tyee {
namespace {

constexpr int kH1 = 32, kH2 = 32;
constexpr int kParams = kH1 * kFeatures + kH1 + kH2 * kH1 + kH2 + kH2 + 1;  // 1377
constexpr int oW1 = 0, oB1 = oW1 + kH1 * kFeatures, oW2 = oB1 + kH1, oB2 = oW2 + kH2 * kH1,
              oW3 = oB2 + kH2, oB3 = oW3 + kH2;
constexpr float kSpan = 0.1f;
constexpr int kBwdEdges = 128;     // edges staged per round of k_mlp_backward
constexpr int kBwdRounds = 32;     // rounds (chunks of kBwdEdges) per block
constexpr int kRow = 139;          // staged floats per edge (138 used, odd stride for LDS banks)

static_assert(kParams == 1377, "parameter count");

// Forward pass of one edge; h1, h2 receive the hidden activations; returns tanh(z).
__device__ __forceinline__ float mlp_edge(const float *__restrict__ P, const float *x, float *h1, float *h2) {
#pragma unroll
    for (int a = 0; a < kH1; ++a) {
        float acc = P[oB1 + a];
#pragma unroll
        for (int b = 0; b < kFeatures; ++b) acc = fmaf(P[oW1 + a * kFeatures + b], x[b], acc);
        h1[a] = tanhf(acc);
    }
#pragma unroll
    for (int a = 0; a < kH2; ++a) {
        float acc = P[oB2 + a];
#pragma unroll
        for (int b = 0; b < kH1; ++b) acc = fmaf(P[oW2 + a * kH1 + b], h1[b], acc);
        h2[a] = tanhf(acc);
    }
    float z = P[oB3];
#pragma unroll
    for (int a = 0; a < kH2; ++a) z = fmaf(P[oW3 + a], h2[a], z);
    return tanhf(z);
}

__device__ __forceinline__ void load_params(float *sP, const float *__restrict__ params) {
    for (int p = threadIdx.x; p < kParams + 2 * kFeatures; p += blockDim.x) sP[p] = params[p];
    __syncthreads();
}

__device__ __forceinline__ void normalise(const float *sP, const float *__restrict__ f, float *x) {
    const float *mu = sP + kParams, *sd = mu + kFeatures;
#pragma unroll
    for (int b = 0; b < kFeatures; ++b) x[b] = (f[b] - mu[b]) / sd[b];
}

// params layout on the device: [1377 model parameters | mu[8] | sd[8]]
__global__ __launch_bounds__(256) void k_mlp_gamma(int n, const float *__restrict__ feat,
                                                   const float *__restrict__ params, float *__restrict__ gamma) {
    __shared__ float sP[kParams + 2 * kFeatures];
    load_params(sP, params);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[kFeatures], h1[kH1], h2[kH2];
    normalise(sP, feat + size_t(i) * kFeatures, x);
    gamma[i] = 1.0f + kSpan * mlp_edge(sP, x, h1, h2);
}

constexpr int kTsThreads = 1024, kTsTris = 4, kTsEdges = 6;  // per work-item
constexpr int kTsMaxTris = kTsThreads * kTsTris, kTsMaxEdges = kTsThreads * kTsEdges;

struct TsMesh {
    int32_t t_off, nt, e_off, ne;
    double dt, area;
};

// One work-group per (mesh m, wave w), b = m * W + w = order[blockIdx.x].
//   tri_word[t][q] = neighbour local triangle | (local edge << 16);  tri_invS, tri_O
//   edge_RL[e] = R | (L << 16) (local triangles);  edge_ebyd = |e|/d;  gamma per edge
__global__ __launch_bounds__(kTsThreads) void k_ts_adjoint(int W, const int32_t *__restrict__ order,
                                                           const TsMesh *__restrict__ meshes,
                                                           const float *__restrict__ waves,
                                                           const int32_t *__restrict__ nsteps,
                                                           const uint32_t *__restrict__ tri_word,
                                                           const float *__restrict__ tri_invS,
                                                           const float *__restrict__ tri_O,
                                                           const uint32_t *__restrict__ edge_RL,
                                                           const float *__restrict__ edge_ebyd,
                                                           const float *__restrict__ gamma, double inv_mw,
                                                           double *__restrict__ eps_out,
                                                           float *__restrict__ grad_out, int64_t grad_stride) {
    // the two sequences' current values, double-buffered: a step reads buffer n & 1 and writes
    // the other, so one barrier per step separates the reads from the next step's writes
    // (real, imaginary) pairs, so that one 8-byte access moves a complex value
    __shared__ float2 lds_state[2][2][kTsMaxTris];
    float2 *xs = lds_state[0][0], *vs = lds_state[0][1];
    auto swap_state = [&](int n) {
        xs = lds_state[n & 1][0];
        vs = lds_state[n & 1][1];
    };
    __shared__ double red[kTsThreads / 64][2];
    // work-groups start longest recurrence first (order sorts (mesh, wave) pairs by steps)
    const int b = order[blockIdx.x];
    const int m = b / W, w = b % W, tid = threadIdx.x;
    const TsMesh M = meshes[m];
    const int N = nsteps[b];
    const float kx = waves[2 * b], kz = waves[2 * b + 1];
    const double kn = sqrt(double(kx) * kx + double(kz) * kz);
    const float dt2 = float(M.dt * M.dt);
    const float ca = float(cos(kn * M.dt / 2)), sa = float(sin(kn * M.dt / 2));

    // own triangles: neighbour words, coupling sigma = gamma^2 |e|/d per side, 1/S
    uint32_t word[kTsTris][3];
    float sig[kTsTris][3], invS[kTsTris];  // sig = -dt^2 gamma^2 (|e|/d) / S per side
    float x_r[kTsTris], x_i[kTsTris], y_r[kTsTris], y_i[kTsTris];
    float v_r[kTsTris], v_i[kTsTris], u_r[kTsTris], u_i[kTsTris];
#pragma unroll
    for (int r = 0; r < kTsTris; ++r) {
        const int t = tid + r * kTsThreads;
        invS[r] = 0.0f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            word[r][q] = 0;
            sig[r][q] = 0.0f;
        }
        x_r[r] = x_i[r] = y_r[r] = y_i[r] = v_r[r] = v_i[r] = u_r[r] = u_i[r] = 0.0f;
        if (t < M.nt) {
            const int g = M.t_off + t;
            invS[r] = tri_invS[g];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const uint32_t wd = tri_word[3 * size_t(g) + q];
                const int e = M.e_off + int(wd >> 16);
                const float ga = gamma[e];
                word[r][q] = wd;
                sig[r][q] = -dt2 * invS[r] * (ga * ga * edge_ebyd[e]);
            }
            // exact wave at t = +dt/2 (x_0) and t = -dt/2 (x_{-1}); y_0 = x_0 - x_{-1}
            const float ph = kx * tri_O[2 * g] + kz * tri_O[2 * g + 1];
            const float br = cosf(ph), bi = sinf(ph);
            x_r[r] = br * ca + bi * sa;     // B e^{-i a}
            x_i[r] = bi * ca - br * sa;
            y_r[r] = 2.0f * bi * sa;        // B (e^{-i a} - e^{i a}) = -2i sin(a) B
            y_i[r] = -2.0f * br * sa;
            v_r[r] = br;                    // v_0 = B, v_{-1} = 0
            v_i[r] = bi;
            u_r[r] = br;
            u_i[r] = bi;
            xs[t] = make_float2(x_r[r], x_i[r]);
            vs[t] = make_float2(v_r[r], v_i[r]);
        }
    }
    __syncthreads();

    // one step of y <- y - dt^2 K s, s <- s + y for the sequences held in (sr, si) / LDS pairs ls
#define TS_STEP(SR, SI, YR, YI, LS)                                                         \
    {                                                                                       \
        float kr = 0.0f, ki = 0.0f;                                                         \
        _Pragma("unroll") for (int q = 0; q < 3; ++q) {                                     \
            const float2 o = LS[int(word[r][q] & 0xFFFFu)];                                 \
            kr = fmaf(sig[r][q], SR[r] - o.x, kr);                                          \
            ki = fmaf(sig[r][q], SI[r] - o.y, ki);                                          \
        }                                                                                   \
        YR[r] += kr;                                                                        \
        YI[r] += ki;                                                                        \
    }

    // pass 1: x and v forward N steps
    for (int n = 0; n < N; ++n) {
        swap_state(n);
#pragma unroll
        for (int r = 0; r < kTsTris; ++r) {
            if (tid + r * kTsThreads < M.nt) {
                TS_STEP(x_r, x_i, y_r, y_i, xs);
                TS_STEP(v_r, v_i, u_r, u_i, vs);
            }
        }
        swap_state(n + 1);
#pragma unroll
        for (int r = 0; r < kTsTris; ++r) {
            const int t = tid + r * kTsThreads;
            if (t < M.nt) {
                x_r[r] += y_r[r];
                x_i[r] += y_i[r];
                v_r[r] += u_r[r];
                v_i[r] += u_i[r];
                xs[t] = make_float2(x_r[r], x_i[r]);
                vs[t] = make_float2(v_r[r], v_i[r]);
            }
        }
        __syncthreads();
    }
    // z_N = sum_j S_j conj(B_j) x_N,j
    double zr = 0.0, zi = 0.0;
#pragma unroll
    for (int r = 0; r < kTsTris; ++r) {
        const int t = tid + r * kTsThreads;
        if (t < M.nt) {
            const int g = M.t_off + t;
            const float ph = kx * tri_O[2 * g] + kz * tri_O[2 * g + 1];
            const double br = cosf(ph), bi = sinf(ph), S = 1.0 / double(invS[r]);
            zr += S * (br * x_r[r] + bi * x_i[r]);
            zi += S * (br * x_i[r] - bi * x_r[r]);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        zr += __shfl_xor(zr, off, 64);
        zi += __shfl_xor(zi, off, 64);
    }
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = zr;
        red[tid >> 6][1] = zi;
    }
    __syncthreads();
    zr = zi = 0.0;
    for (int q = 0; q < kTsThreads / 64; ++q) {
        zr += red[q][0];
        zi += red[q][1];
    }
    // eps = -arg(z_N / z_0) / (|k| N dt) - 1,  z_0 = area e^{-i |k| dt/2}
    const double a0 = kn * M.dt / 2;
    const double qr = zr * cos(a0) - zi * sin(a0), qi = zi * cos(a0) + zr * sin(a0);  // z_N e^{+i a}
    const double T = kn * double(N) * M.dt;
    const double eps = -atan2(qi, qr) / T - 1.0;
    if (tid == 0) eps_out[b] = eps;

    // pass 2: x forward from the start, v backwards from v_{N-1} (u_{N-1} = v_{N-1} - v_N)
#pragma unroll
    for (int r = 0; r < kTsTris; ++r) {
        const int t = tid + r * kTsThreads;
        if (t < M.nt) {
            const float vNr = v_r[r], vNi = v_i[r];
            v_r[r] = vNr - u_r[r];          // v_{N-1}
            v_i[r] = vNi - u_i[r];
            u_r[r] = -u_r[r];
            u_i[r] = -u_i[r];
            const int g = M.t_off + t;
            const float ph = kx * tri_O[2 * g] + kz * tri_O[2 * g + 1];
            const float br = cosf(ph), bi = sinf(ph);
            x_r[r] = br * ca + bi * sa;
            x_i[r] = bi * ca - br * sa;
            y_r[r] = 2.0f * bi * sa;
            y_i[r] = -2.0f * br * sa;
        }
    }
    __syncthreads();   // everyone has read its z-partials before LDS is rewritten
    swap_state(0);
#pragma unroll
    for (int r = 0; r < kTsTris; ++r) {
        const int t = tid + r * kTsThreads;
        if (t < M.nt) {
            xs[t] = make_float2(x_r[r], x_i[r]);
            vs[t] = make_float2(v_r[r], v_i[r]);
        }
    }
    uint32_t erl[kTsEdges];
    float acc_r[kTsEdges], acc_i[kTsEdges];
#pragma unroll
    for (int r = 0; r < kTsEdges; ++r) {
        const int e = tid + r * kTsThreads;
        erl[r] = e < M.ne ? edge_RL[M.e_off + e] : 0u;
        acc_r[r] = acc_i[r] = 0.0f;
    }
    __syncthreads();
    for (int n = 0; n < N; ++n) {
        swap_state(n);
#pragma unroll
        for (int r = 0; r < kTsEdges; ++r) {
            if (tid + r * kTsThreads < M.ne) {
                const int R = int(erl[r] & 0xFFFFu), L = int(erl[r] >> 16);
                const float2 vR = vs[R], vL = vs[L], xR = xs[R], xL = xs[L];
                const float dvr = vR.x - vL.x, dvi = vR.y - vL.y;
                const float dxr = xR.x - xL.x, dxi = xR.y - xL.y;
                acc_r[r] = fmaf(dvr, dxr, fmaf(dvi, dxi, acc_r[r]));   // Re(conj(dv) dx)
                acc_i[r] = fmaf(dvr, dxi, fmaf(-dvi, dxr, acc_i[r]));  // Im(conj(dv) dx)
            }
        }
#pragma unroll
        for (int r = 0; r < kTsTris; ++r) {
            if (tid + r * kTsThreads < M.nt) {
                TS_STEP(x_r, x_i, y_r, y_i, xs);
                TS_STEP(v_r, v_i, u_r, u_i, vs);
            }
        }
        swap_state(n + 1);
#pragma unroll
        for (int r = 0; r < kTsTris; ++r) {
            const int t = tid + r * kTsThreads;
            if (t < M.nt) {
                x_r[r] += y_r[r];
                x_i[r] += y_i[r];
                v_r[r] += u_r[r];
                v_i[r] += u_i[r];
                xs[t] = make_float2(x_r[r], x_i[r]);
                vs[t] = make_float2(v_r[r], v_i[r]);
            }
        }
        __syncthreads();
    }
#undef TS_STEP
    // d eps/d gamma_e = -Im(conj(z_N) dz_e) / |z_N|^2 / T,  dz_e = -2 dt^2 gamma_e (|e|/d) acc_e
    const double zz = zr * zr + zi * zi;
    const double scale = 2.0 * eps * inv_mw / (zz * T);
#pragma unroll
    for (int r = 0; r < kTsEdges; ++r) {
        const int e = tid + r * kTsThreads;
        if (e < M.ne) {
            const int ge = M.e_off + e;
            const double c = -2.0 * M.dt * M.dt * double(gamma[ge]) * double(edge_ebyd[ge]);
            const double dzr = c * acc_r[r], dzi = c * acc_i[r];
            const double im = zr * dzi - zi * dzr;    // Im(conj(z) dz)
            grad_out[size_t(w) * grad_stride + ge] = float(-im * scale);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Multi-work-group form of k_ts_adjoint, for training meshes larger than one work-group's
// LDS.  The two recurrences of every active (mesh, wave) pair live in HBM, one launch per
// step advances every pair that still has steps left (pairs sorted by step count, so the
// active ones are a prefix and form the grid's y dimension), one work-item per triangle:
// it gathers its three neighbours' values of the old buffer and writes its new values to the
// other.  In the second pass the work-item of an edge's R triangle accumulates that edge's
// product conj(v_R - v_L) (x_R - x_L) before the step (each interior edge has one R
// triangle, so no two work-items add to one accumulator).  Every value goes through the same
// single-precision operations in the same order as in k_ts_adjoint, so the two paths give the
// same recurrences; only the FP64 sums of the overlap z_N are added in another order.
// ---------------------------------------------------------------------------------------

struct GtsPair {
    int32_t b, w;           // (mesh, wave) index m * W + w, and the wave
    int32_t t_off, nt;      // the mesh's triangles in the concatenated arrays
    int32_t e_off, ne;      // its edges
    int32_t nsteps;
    int32_t s_off;          // first state entry of this pair (triangles)
    int64_t a_off;          // first accumulator of this pair (edges)
    double dt;
    float kx, kz;
};

constexpr int kGtsThreads = 256;

// sig[g][q] = -dt^2 gamma^2 (|e|/d) / S of each side of the mesh's triangles (as k_ts_adjoint)
__global__ __launch_bounds__(kGtsThreads) void k_gts_coef(int nt, int t_off, int e_off, float dt2,
                                                          const int32_t *__restrict__ side,
                                                          const float *__restrict__ tri_invS,
                                                          const float *__restrict__ edge_ebyd,
                                                          const float *__restrict__ gamma, float *__restrict__ sig) {
    const int j = blockIdx.x * kGtsThreads + threadIdx.x;
    if (j >= nt) return;
    const int g = t_off + j;
    const float invS = tri_invS[g];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int e = e_off + (side[3 * g + q] & 0x7FFFFFFF);
        const float ga = gamma[e];
        sig[3 * size_t(g) + q] = -dt2 * invS * (ga * ga * edge_ebyd[e]);
    }
}

__device__ __forceinline__ void gts_start(const GtsPair &P, const float *__restrict__ tri_O, int g, float2 *x0,
                                          float2 *y0, float2 *v0) {
    const double kn = sqrt(double(P.kx) * P.kx + double(P.kz) * P.kz);
    const float ca = float(cos(kn * P.dt / 2)), sa = float(sin(kn * P.dt / 2));
    const float ph = P.kx * tri_O[2 * g] + P.kz * tri_O[2 * g + 1];
    const float br = cosf(ph), bi = sinf(ph);
    *x0 = make_float2(br * ca + bi * sa, bi * ca - br * sa);
    *y0 = make_float2(2.0f * bi * sa, -2.0f * br * sa);
    *v0 = make_float2(br, bi);
}

// Pass-1 start: x_0, y_0 = x_0 - x_{-1}, v_0 = B, u_0 = v_0 - v_{-1} = B; accumulators zero.
__global__ __launch_bounds__(kGtsThreads) void k_gts_init(const GtsPair *__restrict__ pairs,
                                                          const float *__restrict__ tri_O, float2 *__restrict__ X,
                                                          float2 *__restrict__ Y, float2 *__restrict__ V,
                                                          float2 *__restrict__ U, float2 *__restrict__ acc) {
    const GtsPair P = pairs[blockIdx.y];
    const int j = blockIdx.x * kGtsThreads + threadIdx.x;
    if (j < P.nt) {
        float2 x0, y0, v0;
        gts_start(P, tri_O, P.t_off + j, &x0, &y0, &v0);
        X[P.s_off + j] = x0;
        Y[P.s_off + j] = y0;
        V[P.s_off + j] = v0;
        U[P.s_off + j] = v0;
    }
    if (j < P.ne) acc[P.a_off + j] = make_float2(0.0f, 0.0f);
}

// Pass-2 start: x from the beginning again; v steps backwards from v_{N-1} = v_N - u_N.
__global__ __launch_bounds__(kGtsThreads) void k_gts_mid(const GtsPair *__restrict__ pairs, int64_t buf,
                                                         const float *__restrict__ tri_O, float2 *__restrict__ X,
                                                         float2 *__restrict__ Y, float2 *__restrict__ V,
                                                         float2 *__restrict__ U) {
    const GtsPair P = pairs[blockIdx.y];
    const int j = blockIdx.x * kGtsThreads + threadIdx.x;
    if (j >= P.nt) return;
    const int64_t s = P.s_off + j, last = (P.nsteps & 1) ? buf : 0;  // v_N sits in buffer N & 1
    float2 x0, y0, v0;
    gts_start(P, tri_O, P.t_off + j, &x0, &y0, &v0);
    const float2 vN = V[last + s], uN = U[s];
    X[s] = x0;
    Y[s] = y0;
    V[s] = make_float2(vN.x - uN.x, vN.y - uN.y);
    U[s] = make_float2(-uN.x, -uN.y);
}

// Step n of pass `pass` (1 or 2) for the first gridDim.y pairs (those with n < nsteps).
// X, V: two buffers of `buf` entries each; step n reads buffer n & 1 and writes the other.
__global__ __launch_bounds__(kGtsThreads) void k_gts_step(int n, int pass, int64_t buf,
                                                          const GtsPair *__restrict__ pairs,
                                                          const int32_t *__restrict__ nbr,
                                                          const int32_t *__restrict__ side,
                                                          const float *__restrict__ sig, float2 *__restrict__ X,
                                                          float2 *__restrict__ Y, float2 *__restrict__ V,
                                                          float2 *__restrict__ U, float2 *__restrict__ acc) {
    const GtsPair P = pairs[blockIdx.y];
    const int j = blockIdx.x * kGtsThreads + threadIdx.x;
    if (n >= P.nsteps || j >= P.nt) return;
    const int g = P.t_off + j;
    const int64_t rd = (n & 1) ? buf : 0, wr = (n & 1) ? 0 : buf;
    const float2 *xs = X + rd + P.s_off, *vs = V + rd + P.s_off;
    const float2 xo = xs[j], vo = vs[j];
    int nb[3];
    float2 xn[3], vn[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        nb[q] = nbr[3 * g + q];
        xn[q] = xs[nb[q]];
        vn[q] = vs[nb[q]];
    }
    if (pass == 2) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int sd = side[3 * g + q];
            if (sd < 0) {  // this triangle is R of the edge: L is the neighbour across it
                float2 &a = acc[P.a_off + (sd & 0x7FFFFFFF)];
                const float dvr = vo.x - vn[q].x, dvi = vo.y - vn[q].y;
                const float dxr = xo.x - xn[q].x, dxi = xo.y - xn[q].y;
                float ar = a.x, ai = a.y;
                ar = fmaf(dvr, dxr, fmaf(dvi, dxi, ar));
                ai = fmaf(dvr, dxi, fmaf(-dvi, dxr, ai));
                a = make_float2(ar, ai);
            }
        }
    }
    float kr = 0.0f, ki = 0.0f, lr = 0.0f, li = 0.0f;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const float sg = sig[3 * size_t(g) + q];
        kr = fmaf(sg, xo.x - xn[q].x, kr);
        ki = fmaf(sg, xo.y - xn[q].y, ki);
        lr = fmaf(sg, vo.x - vn[q].x, lr);
        li = fmaf(sg, vo.y - vn[q].y, li);
    }
    const int64_t s = P.s_off + j;
    float2 y = Y[s], u = U[s];
    y.x += kr;
    y.y += ki;
    u.x += lr;
    u.y += li;
    Y[s] = y;
    U[s] = u;
    X[wr + s] = make_float2(xo.x + y.x, xo.y + y.y);
    V[wr + s] = make_float2(vo.x + u.x, vo.y + u.y);
}

// After pass 1: z_N = sum_j S_j conj(B_j) x_N,j per pair (one work-group each, fixed order)
// and eps = -arg(z_N / z_0)/(|k| N dt) - 1.
constexpr int kGtsZThreads = 1024;
__global__ __launch_bounds__(kGtsZThreads) void k_gts_z(const GtsPair *__restrict__ pairs, int64_t buf,
                                                        const float *__restrict__ tri_O,
                                                        const float *__restrict__ tri_invS,
                                                        const float2 *__restrict__ X, double2 *__restrict__ z,
                                                        double *__restrict__ eps_out) {
    __shared__ double red[kGtsZThreads / 64][2];
    const GtsPair P = pairs[blockIdx.x];
    const float2 *xs = X + ((P.nsteps & 1) ? buf : 0) + P.s_off;
    double zr = 0.0, zi = 0.0;
    for (int j = threadIdx.x; j < P.nt; j += kGtsZThreads) {
        const int g = P.t_off + j;
        const float ph = P.kx * tri_O[2 * g] + P.kz * tri_O[2 * g + 1];
        const double br = cosf(ph), bi = sinf(ph), S = 1.0 / double(tri_invS[g]);
        const float2 x = xs[j];
        zr += S * (br * x.x + bi * x.y);
        zi += S * (br * x.y - bi * x.x);
    }
    for (int off = 32; off > 0; off >>= 1) {
        zr += __shfl_xor(zr, off, 64);
        zi += __shfl_xor(zi, off, 64);
    }
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) {
        red[tid >> 6][0] = zr;
        red[tid >> 6][1] = zi;
    }
    __syncthreads();
    if (tid == 0) {
        zr = zi = 0.0;
        for (int q = 0; q < kGtsZThreads / 64; ++q) {
            zr += red[q][0];
            zi += red[q][1];
        }
        const double kn = sqrt(double(P.kx) * P.kx + double(P.kz) * P.kz);
        const double a0 = kn * P.dt / 2;
        const double qr = zr * cos(a0) - zi * sin(a0), qi = zi * cos(a0) + zr * sin(a0);
        const double T = kn * double(P.nsteps) * P.dt;
        z[blockIdx.x] = make_double2(zr, zi);
        eps_out[P.b] = -atan2(qi, qr) / T - 1.0;
    }
}

// After pass 2: the pair's share of dL/dgamma on its mesh's edges (as k_ts_adjoint).
__global__ __launch_bounds__(kGtsThreads) void k_gts_grad(const GtsPair *__restrict__ pairs,
                                                          const double2 *__restrict__ z,
                                                          const double *__restrict__ eps,
                                                          const float2 *__restrict__ acc,
                                                          const float *__restrict__ edge_ebyd,
                                                          const float *__restrict__ gamma, double inv_mw,
                                                          float *__restrict__ grad_out, int64_t grad_stride) {
    const GtsPair P = pairs[blockIdx.y];
    const int e = blockIdx.x * kGtsThreads + threadIdx.x;
    if (e >= P.ne) return;
    const double zr = z[blockIdx.y].x, zi = z[blockIdx.y].y;
    const double kn = sqrt(double(P.kx) * P.kx + double(P.kz) * P.kz);
    const double T = kn * double(P.nsteps) * P.dt;
    const double zz = zr * zr + zi * zi;
    const double scale = 2.0 * eps[P.b] * inv_mw / (zz * T);
    const int ge = P.e_off + e;
    const float2 a = acc[P.a_off + e];
    const double c = -2.0 * P.dt * P.dt * double(gamma[ge]) * double(edge_ebyd[ge]);
    const double dzr = c * a.x, dzi = c * a.y;
    const double im = zr * dzi - zi * dzr;
    grad_out[size_t(P.w) * grad_stride + ge] = float(-im * scale);
}

__global__ void k_fill_f32(int64_t n, float v, float *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}
__global__ void k_fill_f64(int64_t n, double v, double *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// dL/dgamma_e = sum over waves of the per-wave shares (wave order)
__global__ void k_wave_sum(int64_t n, int W, const float *__restrict__ g, float *__restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float acc = 0.0f;
    for (int w = 0; w < W; ++w) acc += g[size_t(w) * n + e];
    out[e] = acc;
}

// Stiff-edge term: beta * mean over the listed edges of (gamma - target)^2.  Edges with a
// tiny dual length barely affect smooth waves but set omega_max (and so dt); pulling their
// gamma below 1 lengthens the stable time step.  One block; adds its gradient to dL/dgamma
// (each listed edge once) and its value to the loss.
__global__ __launch_bounds__(1024) void k_stiff_reg(int count, const int32_t *__restrict__ idx,
                                                    const float *__restrict__ gamma, float beta, float target,
                                                    float *__restrict__ dLdg, double *__restrict__ loss,
                                                    int want_grad) {
    __shared__ double red[1024 / 64];
    double v = 0.0;
    const float inv = 1.0f / float(count > 0 ? count : 1);
    for (int t = threadIdx.x; t < count; t += blockDim.x) {
        const int e = idx[t];
        const float d = gamma[e] - target;
        v += double(beta) * double(d) * double(d) * double(inv);
        if (want_grad) dLdg[e] += 2.0f * beta * d * inv;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int q = 0; q < int(blockDim.x) / 64; ++q) sum += red[q];
        *loss += sum;
    }
}

// loss = sum over the active (mesh, wave) pairs of eps^2 * inv_mw, one block
__global__ __launch_bounds__(1024) void k_loss(int count, const int32_t *__restrict__ active,
                                               const double *__restrict__ eps, double inv_mw,
                                               double *__restrict__ loss) {
    __shared__ double red[1024 / 64];
    double v = 0.0;
    for (int t = threadIdx.x; t < count; t += blockDim.x) {
        const double e = eps[active[t]];
        v += e * e * inv_mw;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < int(blockDim.x) / 64; ++q) s += red[q];
        *loss = s;
    }
}

// Backward pass.  Block b handles edges [b * kBwdEdges * kBwdRounds, ...) in rounds of
// kBwdEdges.  Per round every work-item stages one edge's row
//   [x(8) | h1(32) | d1(32) | h2(32) | d2(32) | dz | 1]
// in LDS; then work-item t accumulates, over the staged rows, the products row[u] * row[v]
// that form the gradient of the parameters it owns (p = t, t + 128, ...).
// idx: the edges to take (n of them, ascending), or null for edges 0 .. n-1.
__global__ __launch_bounds__(kBwdEdges) void k_mlp_backward(int64_t n, const int32_t *__restrict__ idx,
                                                            const float *__restrict__ feat,
                                                            const float *__restrict__ params,
                                                            const float *__restrict__ dLdg,
                                                            float *__restrict__ partial) {
    __shared__ float sP[kParams + 2 * kFeatures];
    __shared__ float rows[kBwdEdges * kRow];
    load_params(sP, params);
    const int t = threadIdx.x;
    constexpr int kOwn = (kParams + kBwdEdges - 1) / kBwdEdges;  // 11
    int16_t u[kOwn], v[kOwn];
    float acc[kOwn];
#pragma unroll
    for (int r = 0; r < kOwn; ++r) {
        const int p = t + r * kBwdEdges;
        int16_t uu = 0, vv = 137;
        if (p < oB1) { uu = int16_t(40 + p / kFeatures); vv = int16_t(p % kFeatures); }
        else if (p < oW2) { uu = int16_t(40 + p - oB1); }
        else if (p < oB2) { uu = int16_t(104 + (p - oW2) / kH1); vv = int16_t(8 + (p - oW2) % kH1); }
        else if (p < oW3) { uu = int16_t(104 + p - oB2); }
        else if (p < oB3) { uu = 136; vv = int16_t(72 + p - oW3); }
        else if (p == oB3) { uu = 136; }
        else { uu = 137; vv = 137; }  // beyond the parameters: unused
        u[r] = uu;
        v[r] = vv;
        acc[r] = 0.0f;
    }
    for (int cc = 0; cc < kBwdRounds; ++cc) {
        const int64_t base = (int64_t(blockIdx.x) * kBwdRounds + cc) * kBwdEdges;
        if (base >= n) break;
        const int cnt = int(n - base < kBwdEdges ? n - base : kBwdEdges);
        __syncthreads();  // previous round's rows fully consumed
        float *row = rows + t * kRow;
        if (t < cnt) {
            const int64_t i = idx ? int64_t(idx[base + t]) : base + t;
            float x[kFeatures], h1[kH1], h2[kH2];
            normalise(sP, feat + size_t(i) * kFeatures, x);
            const float th = mlp_edge(sP, x, h1, h2);
            const float gz = dLdg[i] * kSpan * (1.0f - th * th);  // dL/dz
            float d2[kH2];
#pragma unroll
            for (int a = 0; a < kH2; ++a) d2[a] = gz * sP[oW3 + a] * (1.0f - h2[a] * h2[a]);
#pragma unroll
            for (int b = 0; b < kH1; ++b) {
                float acc1 = 0.0f;
#pragma unroll
                for (int a = 0; a < kH2; ++a) acc1 = fmaf(d2[a], sP[oW2 + a * kH1 + b], acc1);
                row[40 + b] = acc1 * (1.0f - h1[b] * h1[b]);
            }
#pragma unroll
            for (int b = 0; b < kFeatures; ++b) row[b] = x[b];
#pragma unroll
            for (int a = 0; a < kH1; ++a) row[8 + a] = h1[a];
#pragma unroll
            for (int a = 0; a < kH2; ++a) {
                row[72 + a] = h2[a];
                row[104 + a] = d2[a];
            }
            row[136] = gz;
            row[137] = 1.0f;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kOwn; ++r) {
            float a = acc[r];
            for (int e2 = 0; e2 < cnt; ++e2) a = fmaf(rows[e2 * kRow + u[r]], rows[e2 * kRow + v[r]], a);
            acc[r] = a;
        }
    }
#pragma unroll
    for (int r = 0; r < kOwn; ++r) {
        const int p = t + r * kBwdEdges;
        if (p < kParams) partial[size_t(blockIdx.x) * kParams + p] = acc[r];
    }
}

__global__ void k_grad_reduce(int nblocks, const float *__restrict__ partial, float *__restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partial[size_t(b) * kParams + p];
    grad[p] = float(v);
}

__global__ void k_adam(float *__restrict__ params, float *__restrict__ m1, float *__restrict__ m2,
                       const float *__restrict__ grad, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams) return;
    const float g = grad[p];
    const float a = b1 * m1[p] + (1.0f - b1) * g;
    const float b = b2 * m2[p] + (1.0f - b2) * g * g;
    m1[p] = a;
    m2[p] = b;
    params[p] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

template <typename T> int upload_vec(DeviceBuffer &buf, const std::vector<T> &v, hipStream_t s) {
    int rc = buf.alloc(v.size() * sizeof(T));
    if (rc || v.empty()) return rc;
    TYEE_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    TYEE_HIP(hipStreamSynchronize(s));
    return TYEE_OK;
}

template <typename T> int download_vec(const DeviceBuffer &buf, std::vector<T> &v, size_t n, hipStream_t s) {
    v.resize(n);
    if (n == 0) return TYEE_OK;
    TYEE_HIP(hipMemcpyAsync(v.data(), buf.p, n * sizeof(T), hipMemcpyDeviceToHost, s));
    TYEE_HIP(hipStreamSynchronize(s));
    return TYEE_OK;
}

// Overlap of a complex plane-wave state held by two simulations (real and imaginary parts)
// with its initial value: z = sum_i cE_i (Et0_i + i Et1_i) + sum_j cB_j (B0_j + i B1_j), the
// weights cE = (d/gamma) conj(E0) and cB = S conj(B0) in device numbering (metric (7) with
// the scaled edge field).  FP64 partial sums per block, added on the host in block order.
constexpr int kOverlapThreads = 256;

template <typename T>
__global__ __launch_bounds__(kOverlapThreads) void k_overlap(int ne, int nt, const T *__restrict__ Et0,
                                                            const T *__restrict__ Et1, const T *__restrict__ B0,
                                                            const T *__restrict__ B1, const double2 *__restrict__ cE,
                                                            const double2 *__restrict__ cB,
                                                            double *__restrict__ partial) {
    __shared__ double red[2][kOverlapThreads];
    const int i = blockIdx.x * kOverlapThreads + threadIdx.x;
    double zr = 0.0, zi = 0.0;
    if (i < ne) {
        const double a = double(Et0[i]), b = double(Et1[i]);
        const double2 c = cE[i];
        zr += a * c.x - b * c.y;
        zi += a * c.y + b * c.x;
    }
    if (i < nt) {
        const double a = double(B0[i]), b = double(B1[i]);
        const double2 c = cB[i];
        zr += a * c.x - b * c.y;
        zi += a * c.y + b * c.x;
    }
    const int t = threadIdx.x;
    red[0][t] = zr;
    red[1][t] = zi;
    __syncthreads();
    for (int h = kOverlapThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] += red[1][t + h];
        }
        __syncthreads();
    }
    if (t < 2) partial[2 * size_t(blockIdx.x) + t] = red[t][0];
}

template <typename T>
int overlap(Sim &s0, Sim &s1, const DeviceBuffer &cE, const DeviceBuffer &cB, DeviceBuffer &partial, double *zr,
            double *zi) {
    const int64_t n = std::max(s0.ne, s0.nt);
    const int nb = int((n + kOverlapThreads - 1) / kOverlapThreads);
    int rc = partial.alloc(size_t(2) * nb * sizeof(double));
    if (rc) return rc;
    TYEE_HIP(hipStreamSynchronize(s1.stream));
    k_overlap<T><<<nb, kOverlapThreads, 0, s0.stream>>>(int(s0.ne), int(s0.nt), s0.Et().as<T>(), s1.Et().as<T>(),
                                                        s0.B().as<T>(), s1.B().as<T>(), cE.as<double2>(),
                                                        cB.as<double2>(), partial.as<double>());
    TYEE_HIP(hipGetLastError());
    std::vector<double> part;
    rc = download_vec(partial, part, size_t(2) * nb, s0.stream);
    if (rc) return rc;
    *zr = *zi = 0.0;
    for (int b = 0; b < nb; ++b) {
        *zr += part[2 * size_t(b)];
        *zi += part[2 * size_t(b) + 1];
    }
    return TYEE_OK;
}


}  // namespace
}  // namespace tyee

struct tyee_learner {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t M = 0, W = 0, n = 0, nt = 0;  // meshes, waves per mesh, edges, triangles (concatenated)
    tyee::DeviceBuffer feat, ebyd, gamma, waves, nsteps, order, meshes;
    tyee::DeviceBuffer tri_word, tri_invS, tri_O, edge_RL;
    // multi-work-group path: per triangle side its neighbour (local id) and edge (local id,
    // bit 31 set when the triangle is the edge's R), the couplings of the current gamma, the
    // active pairs on that path and their recurrence state and edge accumulators
    tyee::DeviceBuffer g_nbr, g_side, g_sig, g_pairs, g_X, g_Y, g_V, g_U, g_acc, g_z;
    std::vector<tyee::TsMesh> info;         // per mesh (host copy)
    std::vector<int32_t> steps;             // per (mesh, wave)
    std::vector<float> wv;                  // per (mesh, wave) wavevector
    std::vector<uint8_t> fits_lds;          // per mesh: small enough for k_ts_adjoint
    int32_t path = 0;                       // 0 automatic, 1 every mesh on the multi-work-group path
    std::vector<int32_t> active;            // active (mesh, wave) pairs
    std::vector<tyee::GtsPair> gpairs;      // active pairs on the multi-work-group path (steps descending)
    tyee::DeviceBuffer d_active;
    int64_t n_lds_active = 0, g_buf = 0, g_nt_max = 0, g_ne_max = 0;
    tyee::DeviceBuffer bwd_idx;             // edges the MLP backward pass takes under a minibatch
    int64_t n_bwd = 0;
    std::vector<std::vector<int32_t>> stiff_of;  // stiff edges of each mesh
    tyee::DeviceBuffer eps, wave_grad, dLdg, loss, partial_g, grad;
    tyee::DeviceBuffer stiff;            // edges of the stiff-edge term
    int64_t n_stiff = 0;
    double reg_tau = 0.02, reg_beta = 1e-3, reg_target = 0.9;
    std::vector<float> f0;               // d/|e| of every training edge (host)
    tyee::DeviceBuffer params, m1, m2;  // params: [1377 | mu 8 | sd 8]
    int64_t n_bblocks = 0, adam_t = 0;
    std::vector<double> mu, sd;

    ~tyee_learner() {
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

using tyee::fail;

namespace {

// The two passes of the multi-work-group path over its active pairs (see k_gts_step).
int global_pass(tyee_learner &L, double inv_mw, bool want_grad) {
    using namespace tyee;
    hipStream_t s = L.stream;
    const int P = int(L.gpairs.size());
    // couplings of the current gamma, per mesh with an active pair
    std::vector<uint8_t> seen(L.M, 0);
    for (const GtsPair &p : L.gpairs) {
        const int m = p.b / int(L.W);
        if (seen[m]) continue;
        seen[m] = 1;
        const TsMesh &M = L.info[m];
        k_gts_coef<<<(M.nt + kGtsThreads - 1) / kGtsThreads, kGtsThreads, 0, s>>>(
            M.nt, M.t_off, M.e_off, float(M.dt * M.dt), L.g_side.as<int32_t>(), L.tri_invS.as<float>(),
            L.ebyd.as<float>(), L.gamma.as<float>(), L.g_sig.as<float>());
    }
    const int bx_t = int((L.g_nt_max + kGtsThreads - 1) / kGtsThreads);
    const int bx_a = int((std::max(L.g_nt_max, L.g_ne_max) + kGtsThreads - 1) / kGtsThreads);
    const GtsPair *gp = L.g_pairs.as<GtsPair>();
    float2 *X = L.g_X.as<float2>(), *Y = L.g_Y.as<float2>(), *V = L.g_V.as<float2>(), *U = L.g_U.as<float2>();
    float2 *A = L.g_acc.as<float2>();
    k_gts_init<<<dim3(bx_a, P), kGtsThreads, 0, s>>>(gp, L.tri_O.as<float>(), X, Y, V, U, A);
    for (int pass = 1; pass <= (want_grad ? 2 : 1); ++pass) {
        if (pass == 2)
            k_gts_mid<<<dim3(bx_t, P), kGtsThreads, 0, s>>>(gp, L.g_buf, L.tri_O.as<float>(), X, Y, V, U);
        int live = P;
        const int nmax = L.gpairs[0].nsteps;
        for (int n = 0; n < nmax; ++n) {
            while (live > 0 && L.gpairs[live - 1].nsteps <= n) --live;  // steps descending
            k_gts_step<<<dim3(bx_t, live), kGtsThreads, 0, s>>>(n, pass, L.g_buf, gp, L.g_nbr.as<int32_t>(),
                                                                L.g_side.as<int32_t>(), L.g_sig.as<float>(), X,
                                                                Y, V, U, A);
        }
        if (pass == 1)
            k_gts_z<<<P, kGtsZThreads, 0, s>>>(gp, L.g_buf, L.tri_O.as<float>(), L.tri_invS.as<float>(), X,
                                               L.g_z.as<double2>(), L.eps.as<double>());
    }
    if (!want_grad) {
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }
    const int bx_e = int((L.g_ne_max + kGtsThreads - 1) / kGtsThreads);
    k_gts_grad<<<dim3(bx_e, P), kGtsThreads, 0, s>>>(gp, L.g_z.as<double2>(), L.eps.as<double>(), A,
                                                     L.ebyd.as<float>(), L.gamma.as<float>(), inv_mw,
                                                     L.wave_grad.as<float>(), L.n);
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

// Split the active pairs between the two paths, order each by step count (descending) and
// size the multi-work-group state.  Rows of wave_grad that no active pair writes are zeroed
// and the phase errors of inactive pairs set to NaN.
int apply_batch(tyee_learner &L, const std::vector<int32_t> &active) {
    using namespace tyee;
    hipStream_t s = L.stream;
    std::vector<int32_t> lds;
    std::vector<GtsPair> gp;
    for (int32_t b : active) {
        const int m = b / int(L.W), w = b % int(L.W);
        if (L.path == 0 && L.fits_lds[m]) {
            lds.push_back(b);
            continue;
        }
        const TsMesh &M = L.info[m];
        GtsPair p{};
        p.b = b;
        p.w = w;
        p.t_off = M.t_off;
        p.nt = M.nt;
        p.e_off = M.e_off;
        p.ne = M.ne;
        p.nsteps = L.steps[b];
        p.dt = M.dt;
        p.kx = L.wv[2 * size_t(b)];
        p.kz = L.wv[2 * size_t(b) + 1];
        gp.push_back(p);
    }
    std::stable_sort(lds.begin(), lds.end(), [&](int32_t a, int32_t b) { return L.steps[a] > L.steps[b]; });
    std::stable_sort(gp.begin(), gp.end(), [](const GtsPair &a, const GtsPair &b) { return a.nsteps > b.nsteps; });
    int64_t soff = 0, aoff = 0, ntmax = 0, nemax = 0;
    for (GtsPair &p : gp) {
        p.s_off = int32_t(soff);
        p.a_off = aoff;
        soff += p.nt;
        aoff += p.ne;
        ntmax = std::max<int64_t>(ntmax, p.nt);
        nemax = std::max<int64_t>(nemax, p.ne);
    }
    if (soff >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "batch too large for the multi-work-group path");
    // MLP backward edges: every edge of a mesh with an active pair, and the stiff edges of the
    // others (the stiff-edge term covers all training edges), ascending
    std::vector<uint8_t> mesh_on(L.M, 0);
    for (int32_t b : active) mesh_on[b / int(L.W)] = 1;
    std::vector<int32_t> bwd;
    const bool every = std::all_of(mesh_on.begin(), mesh_on.end(), [](uint8_t v) { return v != 0; });
    if (!every) {
        for (int64_t m = 0; m < L.M; ++m) {
            const TsMesh &M = L.info[m];
            if (mesh_on[m]) {
                for (int32_t e = M.e_off; e < M.e_off + M.ne; ++e) bwd.push_back(e);
            } else if (L.reg_beta > 0.0) {
                bwd.insert(bwd.end(), L.stiff_of[m].begin(), L.stiff_of[m].end());
            }
        }
    }
    L.n_bwd = every ? L.n : int64_t(bwd.size());
    L.active = active;
    L.gpairs = gp;
    L.n_lds_active = int64_t(lds.size());
    L.g_buf = soff;
    L.g_nt_max = ntmax;
    L.g_ne_max = nemax;
    int rc = upload_vec(L.d_active, active, s);
    if (!rc && !every) rc = upload_vec(L.bwd_idx, bwd.empty() ? std::vector<int32_t>{0} : bwd, s);
    if (!rc) rc = upload_vec(L.order, lds.empty() ? std::vector<int32_t>{0} : lds, s);
    if (!rc && !gp.empty()) {
        rc = upload_vec(L.g_pairs, gp, s);
        if (!rc) rc = L.g_X.alloc(size_t(2 * soff) * sizeof(float2));
        if (!rc) rc = L.g_V.alloc(size_t(2 * soff) * sizeof(float2));
        if (!rc) rc = L.g_Y.alloc(size_t(soff) * sizeof(float2));
        if (!rc) rc = L.g_U.alloc(size_t(soff) * sizeof(float2));
        if (!rc) rc = L.g_acc.alloc(size_t(aoff) * sizeof(float2));
        if (!rc) rc = L.g_z.alloc(gp.size() * sizeof(double2));
    }
    if (rc) return rc;
    const int64_t ng = L.W * L.n, ne_ = L.M * L.W;
    k_fill_f32<<<int((ng + 255) / 256), 256, 0, s>>>(ng, 0.0f, L.wave_grad.as<float>());
    k_fill_f64<<<int((ne_ + 255) / 256), 256, 0, s>>>(ne_, std::nan(""), L.eps.as<double>());
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

int learner_pass(tyee_learner &L, bool want_grad) {
    using namespace tyee;
    hipStream_t s = L.stream;
    const double inv_mw = 1.0 / double(L.active.size());
    k_mlp_gamma<<<int((L.n + 255) / 256), 256, 0, s>>>(int(L.n), L.feat.as<float>(), L.params.as<float>(),
                                                      L.gamma.as<float>());
    if (L.n_lds_active > 0)
        k_ts_adjoint<<<int(L.n_lds_active), kTsThreads, 0, s>>>(
            int(L.W), L.order.as<int32_t>(), L.meshes.as<TsMesh>(), L.waves.as<float>(), L.nsteps.as<int32_t>(),
            L.tri_word.as<uint32_t>(),
            L.tri_invS.as<float>(), L.tri_O.as<float>(), L.edge_RL.as<uint32_t>(), L.ebyd.as<float>(),
            L.gamma.as<float>(), inv_mw, L.eps.as<double>(), L.wave_grad.as<float>(), L.n);
    if (!L.gpairs.empty()) {
        int rc = global_pass(L, inv_mw, want_grad);
        if (rc) return rc;
    }
    k_loss<<<1, 1024, 0, s>>>(int(L.active.size()), L.d_active.as<int32_t>(), L.eps.as<double>(), inv_mw,
                              L.loss.as<double>());
    if (want_grad)
        // every (mesh, wave) share of dL/dgamma sits in row w of wave_grad; edges of mesh m
        // are touched only by its own W blocks, so the per-edge sum runs over the W rows
        k_wave_sum<<<int((L.n + 255) / 256), 256, 0, s>>>(L.n, int(L.W), L.wave_grad.as<float>(),
                                                          L.dLdg.as<float>());
    if (L.n_stiff > 0 && L.reg_beta > 0.0)
        k_stiff_reg<<<1, 1024, 0, s>>>(int(L.n_stiff), L.stiff.as<int32_t>(), L.gamma.as<float>(),
                                       float(L.reg_beta), float(L.reg_target), L.dLdg.as<float>(),
                                       L.loss.as<double>(), want_grad ? 1 : 0);
    if (want_grad) {
        // with a minibatch only the active meshes' edges and the stiff edges carry a gradient
        const bool list = L.n_bwd < L.n;
        const int64_t nb = (L.n_bwd + kBwdEdges * kBwdRounds - 1) / (kBwdEdges * kBwdRounds);
        k_mlp_backward<<<int(nb), kBwdEdges, 0, s>>>(L.n_bwd, list ? L.bwd_idx.as<int32_t>() : nullptr,
                                                     L.feat.as<float>(), L.params.as<float>(),
                                                     L.dLdg.as<float>(), L.partial_g.as<float>());
        k_grad_reduce<<<(kParams + 255) / 256, 256, 0, s>>>(int(nb), L.partial_g.as<float>(),
                                                            L.grad.as<float>());
    }
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
}

int set_stiff_edges(tyee_learner &L) {
    std::vector<int32_t> idx;
    L.stiff_of.assign(L.M, {});
    for (int64_t m = 0; m < L.M; ++m) {
        const tyee::TsMesh &M = L.info[m];
        for (int32_t e = M.e_off; e < M.e_off + M.ne; ++e)
            if (double(L.f0[e]) < L.reg_tau) {
                idx.push_back(e);
                L.stiff_of[m].push_back(e);
            }
    }
    L.n_stiff = int64_t(idx.size());
    return tyee::upload_vec(L.stiff, idx.empty() ? std::vector<int32_t>{0} : idx, L.stream);
}

int upload_params(tyee_learner &L, const std::vector<double> &theta) {
    std::vector<float> p(tyee::kParams + 2 * tyee::kFeatures);
    for (int k = 0; k < tyee::kParams; ++k) p[k] = float(theta[k]);
    for (int b = 0; b < tyee::kFeatures; ++b) {
        p[tyee::kParams + b] = float(L.mu[b]);
        p[tyee::kParams + tyee::kFeatures + b] = float(L.sd[b]);
    }
    int rc = L.params.alloc(p.size() * sizeof(float));
    if (rc) return rc;
    TYEE_HIP(hipMemcpyAsync(L.params.p, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice, L.stream));
    TYEE_HIP(hipStreamSynchronize(L.stream));
    return TYEE_OK;
}

int current_params(tyee_learner &L, std::vector<double> &theta) {
    std::vector<float> p;
    int rc = tyee::download_vec(L.params, p, tyee::kParams + 2 * tyee::kFeatures, L.stream);
    if (rc) return rc;
    theta.assign(p.begin(), p.begin() + tyee::kParams);
    return TYEE_OK;
}

}  // namespace

extern "C" {

int tyee_learner_create(const tyee_mesh *const *meshes, const double *dt, int64_t n_meshes, const double *waves,
                        int64_t n_waves, double phase, void *stream, tyee_learner **out) {
    using namespace tyee;
    if (!meshes || !dt || !waves || !out || n_meshes <= 0 || n_waves <= 0) return fail(TYEE_EINVAL, "bad learner arguments");
    if (!(phase > 0.0 && phase < 3.0)) return fail(TYEE_EINVAL, "phase must be in (0, 3) radians");
    if (n_meshes * n_waves > (1 << 20)) return fail(TYEE_EINVAL, "too many (mesh, wave) pairs");
    *out = nullptr;
    try {
        std::unique_ptr<tyee_learner> L(new tyee_learner());
        if (stream) {
            L->stream = static_cast<hipStream_t>(stream);
        } else {
            TYEE_HIP(hipStreamCreate(&L->stream));
            L->own_stream = true;
        }
        L->M = n_meshes;
        L->W = n_waves;
        std::vector<float> feat, ebyd, invS, O, wv(2 * n_meshes * n_waves);
        std::vector<uint32_t> word, rl;
        std::vector<int32_t> gnbr, gside;
        std::vector<int32_t> steps(n_meshes * n_waves);
        std::vector<TsMesh> info(n_meshes);
        std::vector<double> sum(kFeatures, 0.0), sum2(kFeatures, 0.0);
        for (int64_t k = 0; k < n_meshes; ++k) {
            if (!meshes[k]) return fail(TYEE_EINVAL, "null mesh");
            const Mesh &m = meshes[k]->m;
            if (!m.periodic) return fail(TYEE_EINVAL, "training meshes must be periodic");
            if (m.nt >= (int64_t(1) << 30) || m.ne >= (int64_t(1) << 30))
                return fail(TYEE_EINVAL, "training mesh too large");
            const bool small = m.nt <= kTsMaxTris && m.ne <= kTsMaxEdges;
            L->fits_lds.push_back(small ? 1 : 0);
            if (!(dt[k] > 0.0)) return fail(TYEE_EINVAL, "dt must be > 0");
            TsMesh &t = info[k];
            t.t_off = int32_t(invS.size());
            t.e_off = int32_t(ebyd.size());
            t.nt = int32_t(m.nt);
            t.ne = int32_t(m.ne);
            t.dt = dt[k];
            t.area = 0.0;
            std::vector<double> f;
            edge_features(m, f);
            for (int64_t i = 0; i < m.ne; ++i) {
                for (int b = 0; b < kFeatures; ++b) {
                    const double x = f[kFeatures * i + b];
                    feat.push_back(float(x));
                    sum[b] += x;
                    sum2[b] += x * x;
                }
                ebyd.push_back(float(m.elen[i] / m.d[i]));
                L->f0.push_back(float(f[kFeatures * i]));
                // 16-bit local triangle ids for the one-work-group kernel (unused above it)
                rl.push_back(small ? uint32_t(m.R[i]) | (uint32_t(m.L[i]) << 16) : 0u);
            }
            for (int64_t j = 0; j < m.nt; ++j) {
                t.area += m.S[j];
                invS.push_back(float(1.0 / m.S[j]));
                O.push_back(float(m.O[2 * j]));
                O.push_back(float(m.O[2 * j + 1]));
                for (int q = 0; q < 3; ++q) {
                    const int32_t i = m.A[3 * j + q];
                    const int32_t nb = m.R[i] == int32_t(j) ? m.L[i] : m.R[i];
                    word.push_back(small ? uint32_t(nb) | (uint32_t(i) << 16) : 0u);
                    gnbr.push_back(nb);
                    gside.push_back(int32_t(uint32_t(i) | (m.R[i] == int32_t(j) ? 0x80000000u : 0u)));
                }
            }
            for (int64_t w = 0; w < n_waves; ++w) {
                const double kx = waves[2 * (k * n_waves + w)], kz = waves[2 * (k * n_waves + w) + 1];
                const double kn = std::hypot(kx, kz);
                if (!(kn > 0.0)) return fail(TYEE_EINVAL, "zero wavevector");
                wv[2 * (k * n_waves + w)] = float(kx);
                wv[2 * (k * n_waves + w) + 1] = float(kz);
                steps[k * n_waves + w] = int32_t(std::max(1.0, std::nearbyint(phase / (kn * dt[k]))));
            }
        }
        L->n = int64_t(ebyd.size());
        L->nt = int64_t(invS.size());
        L->mu.resize(kFeatures);
        L->sd.resize(kFeatures);
        for (int b = 0; b < kFeatures; ++b) {
            L->mu[b] = sum[b] / double(L->n);
            const double var = std::max(0.0, sum2[b] / double(L->n) - L->mu[b] * L->mu[b]);
            L->sd[b] = std::sqrt(var) + 1e-6;
        }
        L->n_bblocks = (L->n + kBwdEdges * kBwdRounds - 1) / (kBwdEdges * kBwdRounds);
        hipStream_t s = L->stream;
        int rc = upload_vec(L->feat, feat, s);
        if (!rc) rc = upload_vec(L->ebyd, ebyd, s);
        if (!rc) rc = upload_vec(L->edge_RL, rl, s);
        if (!rc) rc = upload_vec(L->tri_word, word, s);
        if (!rc) rc = upload_vec(L->tri_invS, invS, s);
        if (!rc) rc = upload_vec(L->tri_O, O, s);
        if (!rc) rc = upload_vec(L->waves, wv, s);
        if (!rc) rc = upload_vec(L->nsteps, steps, s);
        if (!rc) rc = upload_vec(L->g_nbr, gnbr, s);
        if (!rc) rc = upload_vec(L->g_side, gside, s);
        if (!rc) rc = L->g_sig.alloc(gnbr.size() * sizeof(float));
        if (!rc) rc = upload_vec(L->meshes, info, s);
        L->info = info;
        L->steps = steps;
        L->wv = wv;
        if (!rc) rc = L->gamma.alloc(L->n * sizeof(float));
        if (!rc) rc = L->eps.alloc(n_meshes * n_waves * sizeof(double));
        if (!rc) rc = L->wave_grad.alloc(size_t(n_waves) * L->n * sizeof(float));
        if (!rc) rc = L->dLdg.alloc(L->n * sizeof(float));
        if (!rc) rc = L->loss.alloc(sizeof(double));
        if (!rc) rc = L->partial_g.alloc(L->n_bblocks * kParams * sizeof(float));
        if (!rc) rc = L->grad.alloc(kParams * sizeof(float));
        std::vector<float> zeros(kParams, 0.0f);
        if (!rc) rc = upload_vec(L->m1, zeros, s);
        if (!rc) rc = upload_vec(L->m2, zeros, s);
        if (!rc) rc = upload_params(*L, std::vector<double>(kParams, 0.0));
        if (!rc) rc = set_stiff_edges(*L);
        std::vector<int32_t> all(n_meshes * n_waves);
        std::iota(all.begin(), all.end(), 0);
        if (!rc) rc = apply_batch(*L, all);
        if (rc) return rc;
        *out = L.release();
        return TYEE_OK;
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}

int tyee_learner_init(tyee_learner *L, uint64_t seed) {
    using namespace tyee;
    if (!L) return fail(TYEE_EINVAL, "null learner");
    // Glorot-uniform hidden weights from splitmix64, zero biases, zero output layer:
    // the initial model is gamma = 1 on every edge.
    std::vector<double> th(kParams, 0.0);
    auto fill = [&](int o, int fan_out, int fan_in, uint64_t stream_id) {
        const double lim = std::sqrt(6.0 / double(fan_in + fan_out));
        for (int q = 0; q < fan_out * fan_in; ++q) {
            const double u = double(splitmix64(seed + (stream_id << 32) + uint64_t(q)) >> 11) * 0x1.0p-53;
            th[o + q] = (2.0 * u - 1.0) * lim;
        }
    };
    fill(oW1, kH1, kFeatures, 1);
    fill(oW2, kH2, kH1, 2);
    L->adam_t = 0;
    std::vector<float> zeros(kParams, 0.0f);
    int rc = upload_vec(L->m1, zeros, L->stream);
    if (!rc) rc = upload_vec(L->m2, zeros, L->stream);
    return rc ? rc : upload_params(*L, th);
}

int tyee_learner_regulariser(tyee_learner *L, double tau, double beta, double target) {
    if (!L) return fail(TYEE_EINVAL, "null learner");
    if (!(tau >= 0.0) || !(beta >= 0.0) || !(target >= 0.9 && target <= 1.1))
        return fail(TYEE_EINVAL, "tau, beta >= 0 and target in [0.9, 1.1] required");
    L->reg_tau = tau;
    L->reg_beta = beta;
    L->reg_target = target;
    int rc = set_stiff_edges(*L);
    return rc ? rc : apply_batch(*L, L->active);  // the backward edge list follows the stiff edges
}

int tyee_learner_set_params(tyee_learner *L, const double *theta) {
    if (!L || !theta) return fail(TYEE_EINVAL, "null argument");
    return upload_params(*L, std::vector<double>(theta, theta + tyee::kParams));
}

int tyee_learner_get_params(tyee_learner *L, double *theta) {
    if (!L || !theta) return fail(TYEE_EINVAL, "null argument");
    std::vector<double> th;
    int rc = current_params(*L, th);
    if (rc) return rc;
    std::copy(th.begin(), th.end(), theta);
    return TYEE_OK;
}

int tyee_learner_normaliser(tyee_learner *L, const double *mu_in, const double *sd_in, double *mu_out,
                            double *sd_out) {
    if (!L) return fail(TYEE_EINVAL, "null learner");
    if (mu_in && sd_in) {
        for (int b = 0; b < tyee::kFeatures; ++b)
            if (!(sd_in[b] > 0.0)) return fail(TYEE_EINVAL, "feature scales must be > 0");
        std::vector<double> th;
        int rc = current_params(*L, th);
        if (rc) return rc;
        L->mu.assign(mu_in, mu_in + tyee::kFeatures);
        L->sd.assign(sd_in, sd_in + tyee::kFeatures);
        if ((rc = upload_params(*L, th))) return rc;
    }
    if (mu_out) std::copy(L->mu.begin(), L->mu.end(), mu_out);
    if (sd_out) std::copy(L->sd.begin(), L->sd.end(), sd_out);
    return TYEE_OK;
}

int tyee_learner_loss_grad(tyee_learner *L, double *loss, double *grad, double *errors) {
    using namespace tyee;
    if (!L || !loss) return fail(TYEE_EINVAL, "null argument");
    int rc = learner_pass(*L, grad != nullptr);
    if (rc) return rc;
    std::vector<double> l;
    if ((rc = download_vec(L->loss, l, 1, L->stream))) return rc;
    *loss = l[0];
    if (grad) {
        std::vector<float> g;
        if ((rc = download_vec(L->grad, g, kParams, L->stream))) return rc;
        std::copy(g.begin(), g.end(), grad);
    }
    if (errors) {
        std::vector<double> e;
        if ((rc = download_vec(L->eps, e, size_t(L->M * L->W), L->stream))) return rc;
        std::copy(e.begin(), e.end(), errors);
    }
    return TYEE_OK;
}

int tyee_learner_train(tyee_learner *L, int64_t iters, double lr, double *loss_history) {
    using namespace tyee;
    if (!L || iters < 0 || !(lr > 0.0)) return fail(TYEE_EINVAL, "bad training arguments");
    DeviceBuffer hist;
    int rc = hist.alloc(std::max<int64_t>(1, iters) * sizeof(double));
    if (rc) return rc;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int64_t it = 0; it < iters; ++it) {
        if ((rc = learner_pass(*L, true))) return rc;
        TYEE_HIP(hipMemcpyAsync(hist.as<double>() + it, L->loss.p, sizeof(double), hipMemcpyDeviceToDevice,
                                L->stream));
        ++L->adam_t;
        const float c1 = 1.0f - std::pow(b1, float(L->adam_t)), c2 = 1.0f - std::pow(b2, float(L->adam_t));
        k_adam<<<(kParams + 255) / 256, 256, 0, L->stream>>>(L->params.as<float>(), L->m1.as<float>(),
                                                             L->m2.as<float>(), L->grad.as<float>(), float(lr), b1,
                                                             b2, eps, c1, c2);
    }
    TYEE_HIP(hipGetLastError());
    if (loss_history && iters > 0) {
        std::vector<double> h;
        if ((rc = download_vec(hist, h, size_t(iters), L->stream))) return rc;
        std::copy(h.begin(), h.end(), loss_history);
    }
    TYEE_HIP(hipStreamSynchronize(L->stream));
    return TYEE_OK;
}

int tyee_learner_gamma(tyee_learner *L, const tyee_mesh *mesh, double *gamma) {
    using namespace tyee;
    if (!L || !mesh || !gamma) return fail(TYEE_EINVAL, "null argument");
    const Mesh &m = mesh->m;
    std::vector<double> f;
    edge_features(m, f);
    std::vector<float> ff(f.begin(), f.end());
    DeviceBuffer df, dg;
    int rc = upload_vec(df, ff, L->stream);
    if (!rc) rc = dg.alloc(m.ne * sizeof(float));
    if (rc) return rc;
    k_mlp_gamma<<<int((m.ne + 255) / 256), 256, 0, L->stream>>>(int(m.ne), df.as<float>(), L->params.as<float>(),
                                                                dg.as<float>());
    TYEE_HIP(hipGetLastError());
    std::vector<float> g;
    if ((rc = download_vec(dg, g, size_t(m.ne), L->stream))) return rc;
    for (int64_t i = 0; i < m.ne; ++i) gamma[i] = m.interior(i) ? double(g[i]) : 1.0;
    return TYEE_OK;
}

int tyee_learner_set_batch(tyee_learner *L, const int32_t *pairs, int64_t n) {
    if (!L) return fail(TYEE_EINVAL, "null learner");
    std::vector<int32_t> act;
    if (!pairs || n == 0) {
        act.resize(L->M * L->W);
        std::iota(act.begin(), act.end(), 0);
    } else {
        if (n < 0) return fail(TYEE_EINVAL, "negative pair count");
        std::vector<uint8_t> seen(L->M * L->W, 0);
        for (int64_t k = 0; k < n; ++k) {
            const int32_t m = pairs[2 * k], w = pairs[2 * k + 1];
            if (m < 0 || m >= L->M || w < 0 || w >= L->W) return fail(TYEE_EINVAL, "pair out of range");
            const int32_t b = int32_t(m * L->W + w);
            if (seen[b]) return fail(TYEE_EINVAL, "pair listed twice");
            seen[b] = 1;
            act.push_back(b);
        }
    }
    return apply_batch(*L, act);
}

int tyee_learner_set_path(tyee_learner *L, int32_t path) {
    if (!L) return fail(TYEE_EINVAL, "null learner");
    if (path != 0 && path != 1) return fail(TYEE_EINVAL, "path must be 0 (automatic) or 1 (multi-work-group)");
    L->path = path;
    return apply_batch(*L, L->active);
}

void tyee_learner_destroy(tyee_learner *L) { delete L; }

}  // extern "C"

extern "C" int tyee_phase_error_timestepped(const tyee_mesh *mesh, const double *gamma, double dt, int32_t prec,
                                            const double *waves, int64_t n_waves, double phase, int64_t samples,
                                            void *stream, double *eps_out) {
    using namespace tyee;
    if (!mesh || !waves || !eps_out || n_waves <= 0 || !(dt > 0.0) || samples < 2 || !(phase > 0.0))
        return fail(TYEE_EINVAL, "bad phase-error arguments");
    const Mesh &m = mesh->m;
    if (!m.periodic) return fail(TYEE_EINVAL, "plane-wave phase errors need a periodic mesh");
    std::vector<double> w(m.ne, 0.0);
    for (int64_t i = 0; i < m.ne; ++i)
        if (m.interior(i)) w[i] = m.d[i] * m.elen[i];
    // two simulations (real and imaginary parts), created once: the tiles are reused
    tyee_sim *sims[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        tyee_sim_destroy(sims[0]);
        tyee_sim_destroy(sims[1]);
    };
    int rc = TYEE_OK;
    for (int r = 0; r < 2 && !rc; ++r) {
        rc = tyee_sim_create(mesh, prec, dt, stream, &sims[r]);
        if (!rc && gamma) rc = tyee_sim_set_edge_scale(sims[r], gamma);
        if (!rc) rc = tyee_sim_set_fusion(sims[r], 4, 0);
    }
    std::vector<double> Er(m.ne), Ei(m.ne), Br(m.nt), Bi(m.nt);
    DeviceBuffer dcE, dcB, dpart;
    for (int64_t wv = 0; wv < n_waves && !rc; ++wv) {
        const double kx = waves[2 * wv], kz = waves[2 * wv + 1], kn = std::hypot(kx, kz);
        if (!(kn > 0.0)) {
            rc = fail(TYEE_EINVAL, "zero wavevector");
            break;
        }
        // B = exp(i (k.O - |k| dt/2)) at t = dt/2, E = exp(i k.C) (t . (n x k^)) at t = 0
        const double px = -kz / kn, pz = kx / kn;
        for (int64_t j = 0; j < m.nt; ++j) {
            const double ph = kx * m.O[2 * j] + kz * m.O[2 * j + 1] - kn * dt / 2.0;
            Br[j] = std::cos(ph);
            Bi[j] = std::sin(ph);
        }
        for (int64_t i = 0; i < m.ne; ++i) {
            const double ph = kx * m.C[2 * i] + kz * m.C[2 * i + 1];
            const double proj = (m.evec[2 * i] * px + m.evec[2 * i + 1] * pz) / m.elen[i];
            const bool inner = m.interior(i);
            Er[i] = inner ? std::cos(ph) * proj : 0.0;
            Ei[i] = inner ? std::sin(ph) * proj : 0.0;
        }
        for (int r = 0; r < 2 && !rc; ++r) {
            rc = tyee_sim_set_state(sims[r], TYEE_FIELD_E, r ? Ei.data() : Er.data());
            if (!rc) rc = tyee_sim_set_state(sims[r], TYEE_FIELD_B, r ? Bi.data() : Br.data());
        }
        if (rc) break;
        const int64_t nsteps = std::max<int64_t>(samples, int64_t(std::nearbyint(phase / (kn * dt))));
        const int64_t chunk = nsteps / samples;
        double st = 0, sp = 0, stt = 0, stp = 0, prev = 0.0, unwrap = 0.0;
        // overlap weights of this wave in device numbering: (d/gamma) conj(E0), S conj(B0)
        Sim &s0 = sims[0]->s, &s1 = sims[1]->s;
        std::vector<double> cE(2 * m.ne), cB(2 * m.nt);
        for (int64_t k = 0; k < m.ne; ++k) {
            const int32_t i = s0.perm_e[k];
            const double f = m.interior(i) ? w[i] / s0.scale(i) : 0.0;  // d |e| / (gamma |e|)
            cE[2 * k] = f * Er[i];
            cE[2 * k + 1] = -f * Ei[i];
        }
        for (int64_t k = 0; k < m.nt; ++k) {
            const int32_t j = s0.perm_t[k];
            cB[2 * k] = m.S[j] * Br[j];
            cB[2 * k + 1] = -m.S[j] * Bi[j];
        }
        rc = upload_vec(dcE, cE, s0.stream);
        if (!rc) rc = upload_vec(dcB, cB, s0.stream);
        for (int64_t q = 0; q < samples && !rc; ++q) {
            for (int r = 0; r < 2 && !rc; ++r) rc = tyee_sim_step(sims[r], chunk);
            if (rc) break;
            // z = sum w E conj(E0) + sum S B conj(B0)  (metric (7)), reduced on the device
            double zr = 0.0, zi = 0.0;
            rc = s0.f64 ? overlap<double>(s0, s1, dcE, dcB, dpart, &zr, &zi)
                        : overlap<float>(s0, s1, dcE, dcB, dpart, &zr, &zi);
            if (rc) break;
            const double ph = -std::atan2(zi, zr);
            if (q > 0) {
                double dphi = ph - prev;
                while (dphi > M_PI) dphi -= 2.0 * M_PI;
                while (dphi < -M_PI) dphi += 2.0 * M_PI;
                unwrap += dphi;
            } else {
                unwrap = ph;
            }
            prev = ph;
            const double t = double((q + 1) * chunk) * dt;
            st += t;
            sp += unwrap;
            stt += t * t;
            stp += t * unwrap;
        }
        if (rc) break;
        const double n = double(samples);
        eps_out[wv] = (n * stp - st * sp) / (n * stt - st * st) / kn - 1.0;  // least-squares slope
    }
    cleanup();
    return rc;
}

extern "C" int tyee_gate(const tyee_mesh *mesh, const double *gamma, const double *waves, int64_t n_waves,
                         double cfl, double phase, int32_t prec, void *stream, tyee_gate_result *out) {
    using namespace tyee;
    if (!mesh || !gamma || !waves || !out || n_waves <= 0 || !(cfl > 0.0 && cfl < 1.0) ||
        !(phase > 0.0 && phase < 3.0))
        return fail(TYEE_EINVAL, "bad gate arguments");
    const Mesh &m = mesh->m;
    for (int64_t i = 0; i < m.ne; ++i)
        if (!(gamma[i] > 0.0) || !std::isfinite(gamma[i])) return fail(TYEE_EINVAL, "gamma must be > 0");
    tyee_gate_result r{};
    double lp = 0.0, lg = 0.0;
    int64_t ip = 0, ig = 0;
    const int rp = power_iteration(m, nullptr, 20000, 1e-12, 0, &lp, &ip);
    const int rg = power_iteration(m, gamma, 20000, 1e-12, 0, &lg, &ig);
    if ((rp && rp != TYEE_ENOTCONVERGED) || (rg && rg != TYEE_ENOTCONVERGED)) return rp ? rp : rg;
    clear_error();
    r.converged = rp == TYEE_OK && rg == TYEE_OK;
    r.omega_plain = std::sqrt(lp);
    r.omega_learned = std::sqrt(lg);
    r.dt_plain = cfl * 2.0 / r.omega_plain;
    r.dt_learned = cfl * 2.0 / r.omega_learned;
    std::vector<double> ep(n_waves), el(n_waves);
    int rc = tyee_phase_error_timestepped(mesh, nullptr, r.dt_plain, prec, waves, n_waves, phase, 10, stream,
                                          ep.data());
    if (!rc)
        rc = tyee_phase_error_timestepped(mesh, gamma, r.dt_learned, prec, waves, n_waves, phase, 10, stream,
                                          el.data());
    if (rc) return rc;
    for (int64_t w = 0; w < n_waves; ++w) {
        r.err_plain += std::fabs(ep[w]);
        r.err_learned += std::fabs(el[w]);
    }
    r.err_plain /= double(n_waves);
    r.err_learned /= double(n_waves);
    r.accepted = r.converged && r.err_learned < r.err_plain;
    *out = r;
    return TYEE_OK;
}
