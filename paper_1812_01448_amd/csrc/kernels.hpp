// Half-step kernels of the triangular Yee-like leap-frog scheme (arXiv:1812.01448,
// eqs. 3-6) for gfx950. One work-item per cell; every output cell is written by exactly
// one work-item, so no atomics are needed and results do not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tile.hpp"

namespace tyee {

// Sign in bit 31 of a packed edge index: flip the sign bit of the value.
__device__ __forceinline__ float signed_load(const float *__restrict__ v, uint32_t packed) {
    const float x = v[packed & 0x7FFFFFFFu];
    return __uint_as_float(__float_as_uint(x) ^ (packed & 0x80000000u));
}
__device__ __forceinline__ double signed_load(const double *__restrict__ v, uint32_t packed) {
    const double x = v[packed & 0x7FFFFFFFu];
    const unsigned long long bits = __double_as_longlong(x) ^ (uint64_t(packed & 0x80000000u) << 32);
    return __longlong_as_double(bits);
}

// Edge half-step (eq. 3): Et_i += cE_i (B_R - B_L).
template <typename T>
__global__ __launch_bounds__(256) void k_edge(int n, T *__restrict__ Et, const T *__restrict__ B,
                                              const T *__restrict__ cE, const int2 *__restrict__ RL) {
    const int i = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int2 rl = RL[i];
    const T diff = B[rl.x] - B[rl.y];
    Et[i] = fma(cE[i], diff, Et[i]);
}

// Triangle half-step (eq. 4): B_j += nB_j ((s0 Et_0 + s1 Et_1) + s2 Et_2).
template <typename T>
__global__ __launch_bounds__(256) void k_tri(int n, T *__restrict__ B, const T *__restrict__ Et,
                                             const T *__restrict__ nB, const uint32_t *__restrict__ a0,
                                             const uint32_t *__restrict__ a1, const uint32_t *__restrict__ a2) {
    const int j = xcd_group(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const T circ = (signed_load(Et, a0[j]) + signed_load(Et, a1[j])) + signed_load(Et, a2[j]);
    B[j] = fma(nB[j], circ, B[j]);
}

// Plasma current and soft source on the special-edge list (eqs. 5-6), before the edge
// half-step:  jt <- ca jt + cb Et;  delta = dt jt + w g;  Et -= delta.
template <typename T>
__global__ __launch_bounds__(256) void k_special(int n, const int32_t *__restrict__ slot, T *__restrict__ Et,
                                                 T *__restrict__ jt, const T *__restrict__ ca,
                                                 const T *__restrict__ cb, const T *__restrict__ w,
                                                 T *__restrict__ delta, T g, T dt) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int e = slot[k];
    const T e_old = Et[e];
    const T j = fma(ca[k], jt[k], cb[k] * e_old);
    jt[k] = j;
    const T dl = fma(dt, j, w[k] * g);
    delta[k] = dl;
    Et[e] = e_old - dl;
}

// Nodal charge by continuity: Q_v -= sum over its special edges of coef * delta, once per
// step for `steps` consecutive steps whose decrements are stored `stride` apart.  A node
// with up to kChargeRegs incidences keeps them in registers and issues all its decrement
// loads before the arithmetic (the loads are independent; only the sums are ordered); the
// sums run in incidence order either way, so the result does not depend on the path.
constexpr int kChargeRegs = 12;

template <typename T>
__global__ __launch_bounds__(256) void k_charge(int n, const int32_t *__restrict__ node,
                                                const int32_t *__restrict__ off, const int32_t *__restrict__ inc,
                                                const T *__restrict__ coef, const T *__restrict__ delta,
                                                int steps, int stride, T *__restrict__ Q) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int r0 = off[k], deg = off[k + 1] - r0;
    T q = Q[node[k]];
    if (deg <= kChargeRegs) {
        int ii[kChargeRegs];
        T cc[kChargeRegs];
#pragma unroll
        for (int r = 0; r < kChargeRegs; ++r) {
            ii[r] = r < deg ? inc[r0 + r] : 0;
            cc[r] = r < deg ? coef[r0 + r] : T(0);
        }
        for (int s = 0; s < steps; ++s) {
            const T *dl = delta + int64_t(s) * stride;
            T dv[kChargeRegs];
#pragma unroll
            for (int r = 0; r < kChargeRegs; ++r) dv[r] = r < deg ? dl[ii[r]] : T(0);
            T acc = T(0);
#pragma unroll
            for (int r = 0; r < kChargeRegs; ++r)
                if (r < deg) acc = fma(cc[r], dv[r], acc);
            q -= acc;
        }
    } else {
        for (int s = 0; s < steps; ++s) {
            const T *dl = delta + int64_t(s) * stride;
            T acc = T(0);
            for (int r = r0; r < r0 + deg; ++r) acc = fma(coef[r], dl[inc[r]], acc);
            q -= acc;
        }
    }
    Q[node[k]] = q;
}

// Diagnostics (FP64 accumulation): per block, sum of wE Et^2 over edges, sum S B^2 and
// sum S B^{n-1/2} B^{n+1/2} over triangles, max |E| = max |Et| invScale, max |B| and the
// count of non-finite values.  B^{n-1/2} = B^{n+1/2} + (dt/S) ((s0 Et_0 + s1 Et_1) + s2 Et_2)
// undoes the last triangle half-step.  wE = d/(gamma^2 |e|) (0 on outer edges) turns the
// scaled field into metric (7)'s w E^2.  One partial row of 6 doubles per block.
constexpr int kDiagThreads = 256;

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag(int ne, int nt, const T *__restrict__ Et,
                                                      const T *__restrict__ B, const uint32_t *__restrict__ a0,
                                                      const uint32_t *__restrict__ a1, const uint32_t *__restrict__ a2,
                                                      const double *__restrict__ wE, const float *__restrict__ inv_scale,
                                                      const double *__restrict__ S, const double *__restrict__ dtS,
                                                      double *__restrict__ partial) {
    __shared__ double red[6][kDiagThreads];
    const int i = blockIdx.x * kDiagThreads + threadIdx.x;
    double we = 0.0, sb = 0.0, sh = 0.0, me = 0.0, mb = 0.0, bad = 0.0;
    if (i < ne) {
        const double e = double(Et[i]);
        we = wE[i] * e * e;
        me = fabs(e * double(inv_scale[i]));
        bad += isfinite(e) ? 0.0 : 1.0;
    }
    if (i < nt) {
        const double b = double(B[i]);
        const double circ = (double(signed_load(Et, a0[i])) + double(signed_load(Et, a1[i]))) +
                            double(signed_load(Et, a2[i]));
        const double bp = b + dtS[i] * circ;
        sb = S[i] * b * b;
        sh = S[i] * bp * b;
        mb = fabs(b);
        bad += isfinite(b) ? 0.0 : 1.0;
    }
    if (!(me == me)) me = INFINITY;  // NaN never wins a max: record it as infinite
    if (!(mb == mb)) mb = INFINITY;
    const int t = threadIdx.x;
    red[0][t] = we;
    red[1][t] = sb;
    red[2][t] = sh;
    red[3][t] = me;
    red[4][t] = mb;
    red[5][t] = bad;
    __syncthreads();
    for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            red[0][t] += red[0][t + h];
            red[1][t] += red[1][t + h];
            red[2][t] += red[2][t + h];
            red[3][t] = fmax(red[3][t], red[3][t + h]);
            red[4][t] = fmax(red[4][t], red[4][t + h]);
            red[5][t] += red[5][t + h];
        }
        __syncthreads();
    }
    if (t < 6) partial[6 * size_t(blockIdx.x) + t] = red[t][0];
}

// Probe: copy field values at the listed device slots into one row of the sample buffer.
template <typename T>
__global__ __launch_bounds__(256) void k_probe(int n, const int32_t *__restrict__ slot, const T *__restrict__ src,
                                               T *__restrict__ dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[slot[k]];
}

template <typename T>
inline void launch_edge(hipStream_t s, int64_t n, int grid, T *Et, const T *B, const T *cE, const int2 *RL) {
    if (n > 0) k_edge<T><<<grid, 256, 0, s>>>(int(n), Et, B, cE, RL);
}

template <typename T>
inline void launch_tri(hipStream_t s, int64_t n, int grid, T *B, const T *Et, const T *nB, const uint32_t *a0,
                       const uint32_t *a1, const uint32_t *a2) {
    if (n > 0) k_tri<T><<<grid, 256, 0, s>>>(int(n), B, Et, nB, a0, a1, a2);
}

template <typename T>
inline void launch_special(hipStream_t s, int64_t n, const int32_t *slot, T *Et, T *jt, const T *ca, const T *cb,
                           const T *w, T *delta, T g, T dt) {
    if (n > 0) k_special<T><<<int((n + 255) / 256), 256, 0, s>>>(int(n), slot, Et, jt, ca, cb, w, delta, g, dt);
}

template <typename T>
inline void launch_charge(hipStream_t s, int64_t n, const int32_t *node, const int32_t *off, const int32_t *inc,
                          const T *coef, const T *delta, int steps, int stride, T *Q) {
    if (n > 0)
        k_charge<T><<<int((n + 255) / 256), 256, 0, s>>>(int(n), node, off, inc, coef, delta, steps, stride, Q);
}

}  // namespace tyee
