// Learned per-edge coefficient scale for the triangular Yee-like scheme, trained and applied
// on the GPU.
//
// Model: gamma_i = 1 + 0.1 tanh(w3 . tanh(W2 tanh(W1 x_i + b1) + b2) + b3) with
// x_i = (f_i - mu)/sd the normalised eight geometry features of edge i (8 -> 32 -> 32 -> 1,
// 1,377 parameters in the order W1[32][8], b1[32], W2[32][32], b2[32], w3[32], b3).  Scaling
// the eq. 3 and eq. 4 coefficients of an edge by the same gamma keeps metric (7) conserved.
//
// Training signal: the phase error of integer-periodic plane waves exp(i k.O) on training
// meshes.  On a torus |exp(i k.O_j)| = 1, so the Rayleigh quotient of K_gamma = -L_E L_B is
//   omega_RQ^2 = sum_i gamma_i^2 a_i(k) / A,   a_i(k) = (|e_i|/d_i) 4 sin^2(k.(O_R - O_L)/2),
// with A the mesh area; with the leap-frog correction omega = (2/dt) asin(omega_RQ dt/2) the
// error is eps = omega/|k| - 1 and the loss is the mean of eps^2 over meshes and waves.  Its
// gradient in gamma_i is gamma_i sum_w c_w a_i(w) with per-wave coefficients c_w, so one
// pass over the edges gives dL/dgamma, and backpropagation through the MLP gives dL/dtheta.
//
// Kernels (all FP32 arithmetic on edges, FP64 for the per-wave sums and coefficients):
//   k_mlp_gamma     one work-item per edge: the MLP forward pass;
//   k_wave_sums     per chunk of a mesh's edges: partial sums of gamma^2 a(k) for every wave;
//   k_wave_reduce   per (mesh, wave): sum of the chunk partials in chunk order;
//   k_wave_coef     per (mesh, wave): eps, the loss and c_w;
//   k_mlp_backward  per block: forward + backward of its edges, the per-edge activation and
//                   delta vectors staged in LDS, then each work-item accumulates the gradient
//                   of its own parameters over the staged edges (no atomics);
//   k_grad_reduce   per parameter: sum of the block partials in block order;
//   k_adam          per parameter: Adam update.
// Every reduction has a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
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
constexpr int kMaxWaves = 64;
constexpr int kWaveChunk = 4096;   // edges per chunk of k_wave_sums
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

__device__ __forceinline__ float rq_term(float ebyd, float dox, float doz, float kx, float kz) {
    const float s = sinf(0.5f * (kx * dox + kz * doz));
    return ebyd * 4.0f * s * s;
}

// chunk c covers edges [cbeg[c], cend[c]) of mesh cmesh[c]; partial[c][w] = sum gamma^2 a_w.
// Waves are taken in groups of 16 so that the accumulators stay in registers.
__global__ __launch_bounds__(256) void k_wave_sums(const int32_t *__restrict__ cmesh, const int32_t *__restrict__ cbeg,
                                                   const int32_t *__restrict__ cend, int W,
                                                   const float *__restrict__ gamma, const float *__restrict__ ebyd,
                                                   const float *__restrict__ dO, const float *__restrict__ waves,
                                                   double *__restrict__ partial) {
    constexpr int kGroup = 16;
    __shared__ float sk[2 * kMaxWaves];
    __shared__ double red[256 / 64][kGroup];
    const int c = blockIdx.x, m = cmesh[c];
    for (int w = threadIdx.x; w < 2 * W; w += blockDim.x) sk[w] = waves[2 * size_t(m) * W + w];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int g0 = 0; g0 < W; g0 += kGroup) {
        float acc[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) acc[q] = 0.0f;
        for (int i = cbeg[c] + threadIdx.x; i < cend[c]; i += blockDim.x) {
            const float g2 = gamma[i] * gamma[i], e = ebyd[i], dx = dO[2 * i], dz = dO[2 * i + 1];
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const int w = g0 + q;
                if (w < W) acc[q] = fmaf(g2, rq_term(e, dx, dz, sk[2 * w], sk[2 * w + 1]), acc[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            double v = acc[q];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) red[wv][q] = v;
        }
        __syncthreads();
        if (threadIdx.x < kGroup && g0 + int(threadIdx.x) < W) {
            double v = 0.0;
            for (int q = 0; q < int(blockDim.x) / 64; ++q) v += red[q][threadIdx.x];
            partial[size_t(c) * W + g0 + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

// S[m][w] = sum over the chunks of mesh m (chunks of a mesh are consecutive)
__global__ void k_wave_reduce(int M, int W, const int32_t *__restrict__ mesh_chunk0, const double *__restrict__ partial,
                              double *__restrict__ S) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * W) return;
    const int m = t / W, w = t % W;
    double v = 0.0;
    for (int c = mesh_chunk0[m]; c < mesh_chunk0[m + 1]; ++c) v += partial[size_t(c) * W + w];
    S[t] = v;
}

// eps, loss and gradient coefficient c_w for every (mesh, wave); one block
__global__ __launch_bounds__(1024) void k_wave_coef(int M, int W, const double *__restrict__ S,
                                                    const double *__restrict__ area, const double *__restrict__ dt,
                                                    const float *__restrict__ waves, double *__restrict__ eps,
                                                    float *__restrict__ coef, double *__restrict__ loss_out) {
    __shared__ double red[1024 / 64];
    const double inv = 1.0 / double(M * W);
    double local = 0.0;
    for (int t = threadIdx.x; t < M * W; t += blockDim.x) {
        const int m = t / W;
        const double kx = waves[2 * t], kz = waves[2 * t + 1];
        const double kn = sqrt(kx * kx + kz * kz);
        const double wrq = sqrt(S[t] / area[m]);
        const double s = wrq * dt[m] / 2.0;
        const double e = 2.0 / dt[m] * asin(s) / kn - 1.0;
        eps[t] = e;
        local += e * e * inv;
        // dL/dgamma_i = gamma_i sum_w c_w a_i(w)
        coef[t] = float(2.0 * e * inv / (kn * sqrt(1.0 - s * s)) / (area[m] * wrq));
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int q = 0; q < int(blockDim.x) / 64; ++q) v += red[q];
        *loss_out = v;
    }
}

// Backward pass.  Block b handles backward chunks [b*kBwdRounds, (b+1)*kBwdRounds) of at most
// kBwdEdges edges of one mesh each.  Per chunk every work-item stages one edge's row
//   [x(8) | h1(32) | d1(32) | h2(32) | d2(32) | dz | 1]
// in LDS; then work-item t accumulates, over the staged rows, the products row[u] * row[v]
// that form the gradient of the parameters it owns (p = t, t + 128, ...).
__global__ __launch_bounds__(kBwdEdges) void k_mlp_backward(int nchunks, const int32_t *__restrict__ cmesh,
                                                            const int32_t *__restrict__ cbeg,
                                                            const int32_t *__restrict__ cend, int W,
                                                            const float *__restrict__ feat,
                                                            const float *__restrict__ params,
                                                            const float *__restrict__ ebyd,
                                                            const float *__restrict__ dO,
                                                            const float *__restrict__ waves,
                                                            const float *__restrict__ coef,
                                                            float *__restrict__ partial) {
    __shared__ float sP[kParams + 2 * kFeatures];
    __shared__ float rows[kBwdEdges * kRow];
    __shared__ float sw[3 * kMaxWaves];
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
        const int c = blockIdx.x * kBwdRounds + cc;
        if (c >= nchunks) break;
        const int m = cmesh[c], i = cbeg[c] + t, n = cend[c] - cbeg[c];
        __syncthreads();  // previous round's rows fully consumed
        for (int w = t; w < W; w += blockDim.x) {
            sw[3 * w] = waves[2 * (size_t(m) * W + w)];
            sw[3 * w + 1] = waves[2 * (size_t(m) * W + w) + 1];
            sw[3 * w + 2] = coef[size_t(m) * W + w];
        }
        __syncthreads();
        float *row = rows + t * kRow;
        if (t < n) {
            float x[kFeatures], h1[kH1], h2[kH2];
            normalise(sP, feat + size_t(i) * kFeatures, x);
            const float th = mlp_edge(sP, x, h1, h2);
            const float gam = 1.0f + kSpan * th;
            // dL/dgamma_i
            const float e = ebyd[i], dx = dO[2 * i], dz = dO[2 * i + 1];
            float s = 0.0f;
            for (int w = 0; w < W; ++w) s = fmaf(sw[3 * w + 2], rq_term(e, dx, dz, sw[3 * w], sw[3 * w + 1]), s);
            const float gz = gam * s * kSpan * (1.0f - th * th);  // dL/dz
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
            for (int e2 = 0; e2 < n; ++e2) a = fmaf(rows[e2 * kRow + u[r]], rows[e2 * kRow + v[r]], a);
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

}  // namespace
}  // namespace tyee

struct tyee_learner {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t M = 0, W = 0, n = 0;  // meshes, waves per mesh, edges (interior, concatenated)
    tyee::DeviceBuffer feat, ebyd, dO, gamma, waves, area, dt;
    tyee::DeviceBuffer wc_mesh, wc_beg, wc_end, mesh_chunk0, partial_w, S, eps, coef, loss;
    tyee::DeviceBuffer bc_mesh, bc_beg, bc_end, partial_g, grad;
    tyee::DeviceBuffer params, m1, m2;  // params: [1377 | mu 8 | sd 8]
    int64_t n_wchunks = 0, n_bchunks = 0, n_bblocks = 0, adam_t = 0;
    std::vector<double> mu, sd;

    ~tyee_learner() {
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

using tyee::fail;

namespace {

int learner_pass(tyee_learner &L, bool want_grad) {
    using namespace tyee;
    const int M = int(L.M), W = int(L.W);
    hipStream_t s = L.stream;
    k_mlp_gamma<<<int((L.n + 255) / 256), 256, 0, s>>>(int(L.n), L.feat.as<float>(), L.params.as<float>(),
                                                      L.gamma.as<float>());
    k_wave_sums<<<int(L.n_wchunks), 256, 0, s>>>(L.wc_mesh.as<int32_t>(), L.wc_beg.as<int32_t>(),
                                                 L.wc_end.as<int32_t>(), W, L.gamma.as<float>(),
                                                 L.ebyd.as<float>(), L.dO.as<float>(), L.waves.as<float>(),
                                                 L.partial_w.as<double>());
    k_wave_reduce<<<(M * W + 255) / 256, 256, 0, s>>>(M, W, L.mesh_chunk0.as<int32_t>(), L.partial_w.as<double>(),
                                                      L.S.as<double>());
    k_wave_coef<<<1, 1024, 0, s>>>(M, W, L.S.as<double>(), L.area.as<double>(), L.dt.as<double>(),
                                   L.waves.as<float>(), L.eps.as<double>(), L.coef.as<float>(),
                                   L.loss.as<double>());
    if (want_grad) {
        k_mlp_backward<<<int(L.n_bblocks), kBwdEdges, 0, s>>>(
            int(L.n_bchunks), L.bc_mesh.as<int32_t>(), L.bc_beg.as<int32_t>(), L.bc_end.as<int32_t>(), W,
            L.feat.as<float>(), L.params.as<float>(), L.ebyd.as<float>(), L.dO.as<float>(), L.waves.as<float>(),
            L.coef.as<float>(), L.partial_g.as<float>());
        k_grad_reduce<<<(kParams + 255) / 256, 256, 0, s>>>(int(L.n_bblocks), L.partial_g.as<float>(),
                                                            L.grad.as<float>());
    }
    TYEE_HIP(hipGetLastError());
    return TYEE_OK;
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
                        int64_t n_waves, void *stream, tyee_learner **out) {
    using namespace tyee;
    if (!meshes || !dt || !waves || !out || n_meshes <= 0 || n_waves <= 0) return fail(TYEE_EINVAL, "bad learner arguments");
    if (n_waves > kMaxWaves) return fail(TYEE_EINVAL, "at most 64 waves per mesh");
    if (n_meshes * n_waves > 1 << 20) return fail(TYEE_EINVAL, "too many (mesh, wave) pairs");
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
        std::vector<float> feat, ebyd, dO;
        std::vector<double> area(n_meshes), dts(dt, dt + n_meshes);
        std::vector<int32_t> wc_mesh, wc_beg, wc_end, chunk0{0}, bc_mesh, bc_beg, bc_end;
        std::vector<double> sum(kFeatures, 0.0), sum2(kFeatures, 0.0);
        int64_t off = 0;
        for (int64_t k = 0; k < n_meshes; ++k) {
            if (!meshes[k]) return fail(TYEE_EINVAL, "null mesh");
            const Mesh &m = meshes[k]->m;
            if (!(dt[k] > 0.0)) return fail(TYEE_EINVAL, "dt must be > 0");
            std::vector<double> f, dv;
            edge_features(m, f);
            dual_vectors(m, dv);
            const int64_t start = off;
            for (int64_t i = 0; i < m.ne; ++i) {
                if (!m.interior(i)) continue;
                for (int b = 0; b < kFeatures; ++b) {
                    const double x = f[kFeatures * i + b];
                    feat.push_back(float(x));
                    sum[b] += x;
                    sum2[b] += x * x;
                }
                ebyd.push_back(float(m.elen[i] / m.d[i]));
                dO.push_back(float(dv[2 * i]));
                dO.push_back(float(dv[2 * i + 1]));
                ++off;
            }
            for (int64_t c = start; c < off; c += kWaveChunk) {
                wc_mesh.push_back(int32_t(k));
                wc_beg.push_back(int32_t(c));
                wc_end.push_back(int32_t(std::min<int64_t>(off, c + kWaveChunk)));
            }
            chunk0.push_back(int32_t(wc_mesh.size()));
            for (int64_t c = start; c < off; c += kBwdEdges) {
                bc_mesh.push_back(int32_t(k));
                bc_beg.push_back(int32_t(c));
                bc_end.push_back(int32_t(std::min<int64_t>(off, c + kBwdEdges)));
            }
            double a = 0.0;
            for (int64_t j = 0; j < m.nt; ++j) a += m.S[j];
            area[k] = a;
        }
        L->n = off;
        if (off == 0 || off > INT32_MAX) return fail(TYEE_EINVAL, "no interior edges");
        L->mu.resize(kFeatures);
        L->sd.resize(kFeatures);
        for (int b = 0; b < kFeatures; ++b) {
            L->mu[b] = sum[b] / double(off);
            const double var = std::max(0.0, sum2[b] / double(off) - L->mu[b] * L->mu[b]);
            L->sd[b] = std::sqrt(var) + 1e-6;
        }
        std::vector<float> wv(2 * n_meshes * n_waves);
        for (size_t q = 0; q < wv.size(); ++q) wv[q] = float(waves[q]);
        L->n_wchunks = int64_t(wc_mesh.size());
        L->n_bchunks = int64_t(bc_mesh.size());
        L->n_bblocks = (L->n_bchunks + kBwdRounds - 1) / kBwdRounds;
        hipStream_t s = L->stream;
        int rc = upload_vec(L->feat, feat, s);
        if (!rc) rc = upload_vec(L->ebyd, ebyd, s);
        if (!rc) rc = upload_vec(L->dO, dO, s);
        if (!rc) rc = L->gamma.alloc(off * sizeof(float));
        if (!rc) rc = upload_vec(L->waves, wv, s);
        if (!rc) rc = upload_vec(L->area, area, s);
        if (!rc) rc = upload_vec(L->dt, dts, s);
        if (!rc) rc = upload_vec(L->wc_mesh, wc_mesh, s);
        if (!rc) rc = upload_vec(L->wc_beg, wc_beg, s);
        if (!rc) rc = upload_vec(L->wc_end, wc_end, s);
        if (!rc) rc = upload_vec(L->mesh_chunk0, chunk0, s);
        if (!rc) rc = L->partial_w.alloc(L->n_wchunks * n_waves * sizeof(double));
        if (!rc) rc = L->S.alloc(n_meshes * n_waves * sizeof(double));
        if (!rc) rc = L->eps.alloc(n_meshes * n_waves * sizeof(double));
        if (!rc) rc = L->coef.alloc(n_meshes * n_waves * sizeof(float));
        if (!rc) rc = L->loss.alloc(sizeof(double));
        if (!rc) rc = upload_vec(L->bc_mesh, bc_mesh, s);
        if (!rc) rc = upload_vec(L->bc_beg, bc_beg, s);
        if (!rc) rc = upload_vec(L->bc_end, bc_end, s);
        if (!rc) rc = L->partial_g.alloc(L->n_bblocks * kParams * sizeof(float));
        if (!rc) rc = L->grad.alloc(kParams * sizeof(float));
        std::vector<float> zeros(kParams, 0.0f);
        if (!rc) rc = upload_vec(L->m1, zeros, s);
        if (!rc) rc = upload_vec(L->m2, zeros, s);
        if (!rc) rc = upload_params(*L, std::vector<double>(kParams, 0.0));
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

void tyee_learner_destroy(tyee_learner *L) { delete L; }

}  // extern "C"

extern "C" int tyee_phase_error_timestepped(const tyee_mesh *mesh, const double *gamma, double dt, int32_t prec,
                                            double kx, double kz, int64_t nsteps, int64_t samples, void *stream,
                                            double *eps_out) {
    using namespace tyee;
    if (!mesh || !eps_out || !(dt > 0.0) || nsteps <= 0 || samples < 2 || samples > nsteps)
        return fail(TYEE_EINVAL, "bad phase-error arguments");
    const double kn = std::hypot(kx, kz);
    if (!(kn > 0.0)) return fail(TYEE_EINVAL, "zero wavevector");
    const Mesh &m = mesh->m;
    // complex plane wave: B = exp(i (k.O - |k| dt/2)) at t = dt/2, E = exp(i k.C) (t . (n x k^)) at t = 0
    std::vector<double> Er(m.ne), Ei(m.ne), Br(m.nt), Bi(m.nt), w(m.ne, 0.0);
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
        if (inner) w[i] = m.d[i] * m.elen[i];
    }
    tyee_sim *sims[2] = {nullptr, nullptr};
    auto cleanup = [&]() {
        tyee_sim_destroy(sims[0]);
        tyee_sim_destroy(sims[1]);
    };
    int rc = TYEE_OK;
    for (int r = 0; r < 2 && !rc; ++r) {
        rc = tyee_sim_create(mesh, prec, dt, stream, &sims[r]);
        if (!rc && gamma) rc = tyee_sim_set_edge_scale(sims[r], gamma);
        if (!rc) rc = tyee_sim_set_state(sims[r], TYEE_FIELD_E, r ? Ei.data() : Er.data());
        if (!rc) rc = tyee_sim_set_state(sims[r], TYEE_FIELD_B, r ? Bi.data() : Br.data());
        if (!rc) rc = tyee_sim_set_fusion(sims[r], 4, 0);
    }
    if (rc) {
        cleanup();
        return rc;
    }
    const int64_t chunk = nsteps / samples;
    std::vector<double> ts, phase;
    std::vector<double> E[2], B[2];
    double prev = 0.0, unwrap = 0.0;
    for (int64_t q = 0; q < samples && !rc; ++q) {
        for (int r = 0; r < 2 && !rc; ++r) {
            rc = tyee_sim_step(sims[r], chunk);
            E[r].resize(m.ne);
            B[r].resize(m.nt);
            if (!rc) rc = tyee_sim_get_state(sims[r], TYEE_FIELD_E, E[r].data());
            if (!rc) rc = tyee_sim_get_state(sims[r], TYEE_FIELD_B, B[r].data());
        }
        if (rc) break;
        // z = sum w E conj(E0) + sum S B conj(B0)
        double zr = 0.0, zi = 0.0;
        for (int64_t i = 0; i < m.ne; ++i) {
            zr += w[i] * (E[0][i] * Er[i] + E[1][i] * Ei[i]);
            zi += w[i] * (E[1][i] * Er[i] - E[0][i] * Ei[i]);
        }
        for (int64_t j = 0; j < m.nt; ++j) {
            zr += m.S[j] * (B[0][j] * Br[j] + B[1][j] * Bi[j]);
            zi += m.S[j] * (B[1][j] * Br[j] - B[0][j] * Bi[j]);
        }
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
        ts.push_back(double((q + 1) * chunk) * dt);
        phase.push_back(unwrap);
    }
    cleanup();
    if (rc) return rc;
    // least-squares slope of phase(t)
    const double n = double(ts.size());
    double st = 0, sp = 0, stt = 0, stp = 0;
    for (size_t q = 0; q < ts.size(); ++q) {
        st += ts[q];
        sp += phase[q];
        stt += ts[q] * ts[q];
        stp += ts[q] * phase[q];
    }
    const double slope = (n * stp - st * sp) / (n * stt - st * st);
    *eps_out = slope / kn - 1.0;
    return TYEE_OK;
}
