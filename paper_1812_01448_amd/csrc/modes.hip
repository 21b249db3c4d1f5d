// Lowest (or highest) eigenmodes of the B-field operator K = -L_E L_B (Section 2: eigenvectors
// of the Maxwell operator in metric (7) and the "complex time" method), on the device in FP64.
// The highest modes are the lowest of b - K (b the bound below), which the same iteration finds.
//
// With E eliminated, eqs. 3-4 give for the field at triangle j
//     (K B)_j = (1/S_j) sum over interior edges i of j of  w_i (B_j - B_other(i)),
//     w_i = gamma_i^2 |e_i| / d_i,
// a weighted Laplacian of the dual graph that is self-adjoint and non-negative in the B part
// of metric (7) (weights S_j).  Its eigenpairs K v = lambda v give the resonator modes,
// omega = sqrt(lambda); the constant field is the static mode (lambda = 0).
//
// The paper iterates the leap-frog system in imaginary time, normalising every step, so that
// the mode with the largest eigenvalue outgrows the others, and removes found modes by
// orthogonality in metric (7).  Here that idea is aimed at the low end of the spectrum and
// run on a block of vectors:
//   * filter: the three-term recurrence y_{k+1} = 2 x(K) y_k - y_{k-1} is the leap-frog of
//     eqs. 3-4 with E eliminated.  Shifting and scaling K so that the unwanted part of the
//     spectrum [a, b] maps to [-1, 1] puts those modes inside the stability bound of eq. 20:
//     they oscillate with bounded amplitude, while the wanted modes below a violate the bound
//     and grow exponentially (the complex-time amplification).  The recurrence is the scaled
//     Chebyshev filter of Zhou and Saad (J. Comput. Phys. 2007), which keeps the block in
//     range;
//   * deflation: the filtered block is made S-orthonormal (Cholesky QR twice; the shifted
//     CholeskyQR3 of Fukaya et al., SIAM J. Sci. Comput. 2020, when a factorisation fails), so
//     every vector is orthogonal in metric (7) to the others;
//   * Rayleigh-Ritz: H = V^T S K V is diagonalised (cyclic Jacobi) and V rotated into Ritz
//     vectors; the largest Ritz value of the block becomes the next a.
// An outer iteration runs three filter passes, each followed by the orthonormalisation (subspace
// iteration needs no Rayleigh-Ritz in between; before another pass one Cholesky QR, which
// leaves the block well conditioned, is enough), then one Rayleigh-Ritz step.
// b is a Gershgorin bound on lambda_max of the symmetric form S^(1/2) K S^(-1/2).
//
// Layout: the block is row-major, [n_t][nb] doubles (row = triangle in device numbering), so
// the three neighbour rows that a triangle gathers are contiguous runs of nb values.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <utility>
#include <vector>

#include "sim.hpp"

namespace tyee {
namespace {

constexpr int kMaxBlock = 256;
typedef double double4v __attribute__((ext_vector_type(4)));   // one lane's share of a 16 x 16 FP64 MFMA tile
constexpr int kJacobiSweeps = 40;   // sweep limit of the Rayleigh-Ritz eigensolver
constexpr int kStartSweeps = 3;     // the same for the random starting block
constexpr int kMidSweeps = 3;       // the same while the residuals are far from the tolerance
constexpr double kNearTol = 1e4;    // "far": above kNearTol x the tolerance
constexpr int kFilterPasses = 3;    // filter + Cholesky QR passes per Rayleigh-Ritz step

// y_out = alpha * (K y) + beta * y + gam * y_prev   (y_prev may be null).  One wave per row
// (triangle): the row's neighbour slots, weights and 1/S are wave-uniform (scalar loads) and
// the lanes walk its nb columns, so the three neighbour rows are read as contiguous runs.
// Work-groups are remapped so that each XCD takes one contiguous run of rows: a row's
// neighbours (close in the locality numbering) are then gathered through the same XCD's L2.
constexpr int kApplyWaves = 4;  // rows per work-group of the apply kernel
template <int CH>                // 64-column chunks per row: ceil(nb / 64)
__global__ void __launch_bounds__(64 * kApplyWaves) k_modes_apply(
    int32_t n, int32_t nb, const double *__restrict__ y, const double *__restrict__ yp, double *__restrict__ yo,
    const int32_t *__restrict__ nbr, const double *__restrict__ wt, const double *__restrict__ inv_s, double alpha,
    double beta, double gam) {
    const int j = __builtin_amdgcn_readfirstlane(xcd_group(blockIdx.x, gridDim.x) * kApplyWaves +
                                                 int(threadIdx.x >> 6));
    if (j >= n) return;
    const int lane = threadIdx.x & 63;
    int32_t o[3];
    double w[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o[q] = nbr[3 * j + q];
        w[q] = wt[3 * j + q];
    }
    const double is = inv_s[j];
    const size_t row = size_t(j) * nb;
    // all loads of the row first (columns past nb read column nb - 1, and a missing neighbour
    // reads the row itself: valid addresses whose values are not used), then the updates
    double yv[CH], g[CH][3], pv[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = min(lane + 64 * k, nb - 1);
        yv[k] = y[row + c];
#pragma unroll
        for (int q = 0; q < 3; ++q) g[k][q] = y[size_t(o[q] >= 0 ? o[q] : j) * nb + c];
        pv[k] = yp ? yp[row + c] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = lane + 64 * k;
        if (c >= nb) break;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (o[q] >= 0) acc += w[q] * (yv[k] - g[k][q]);
        double out = alpha * (acc * is) + beta * yv[k];
        if (yp) out += gam * pv[k];
        yo[row + c] = out;
    }
}

// The same for an even nb, two columns per work-item (16-byte loads and stores; rows are
// 16-byte aligned): CH2 chunks of 128 columns per row.
template <int CH2>               // ceil(nb / 128)
__global__ void __launch_bounds__(64 * kApplyWaves) k_modes_apply2(
    int32_t n, int32_t nb, const double *__restrict__ y, const double *__restrict__ yp, double *__restrict__ yo,
    const int32_t *__restrict__ nbr, const double *__restrict__ wt, const double *__restrict__ inv_s, double alpha,
    double beta, double gam) {
    const int j = __builtin_amdgcn_readfirstlane(xcd_group(blockIdx.x, gridDim.x) * kApplyWaves +
                                                 int(threadIdx.x >> 6));
    if (j >= n) return;
    const int lane = threadIdx.x & 63, h2 = nb >> 1;
    int32_t o[3];
    double w[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o[q] = nbr[3 * j + q];
        w[q] = wt[3 * j + q];
    }
    const double is = inv_s[j];
    const double2 *y2 = reinterpret_cast<const double2 *>(y), *p2 = reinterpret_cast<const double2 *>(yp);
    double2 *o2 = reinterpret_cast<double2 *>(yo);
    const size_t row = size_t(j) * h2;
    double2 yv[CH2], g[CH2][3], pv[CH2];
#pragma unroll
    for (int k = 0; k < CH2; ++k) {
        const int c = min(lane + 64 * k, h2 - 1);
        yv[k] = y2[row + c];
#pragma unroll
        for (int q = 0; q < 3; ++q) g[k][q] = y2[size_t(o[q] >= 0 ? o[q] : j) * h2 + c];
        pv[k] = yp ? p2[row + c] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < CH2; ++k) {
        const int c = lane + 64 * k;
        if (c >= h2) break;
        double ax = 0.0, ay = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (o[q] >= 0) {
                ax += w[q] * (yv[k].x - g[k][q].x);
                ay += w[q] * (yv[k].y - g[k][q].y);
            }
        double ox = alpha * (ax * is) + beta * yv[k].x, oy = alpha * (ay * is) + beta * yv[k].y;
        if (yp) {
            ox += gam * pv[k].x;
            oy += gam * pv[k].y;
        }
        o2[row + c] = make_double2(ox, oy);
    }
}

// y_out = alpha * ((K - sigma)^2 y) + beta * y + gam * y_prev (y_prev may be null), in one pass:
// row j of (K - sigma)^2 y needs (K - sigma) y at j and at its neighbours k, and those need the
// neighbours of k, so a wave (one row) reads up to ten rows of y (the two-ring of j, mostly
// from the caches: neighbouring rows are close in the locality numbering; row j, which is in
// each neighbour's ring, is read once).  The weights,
// neighbour slots and 1/S of the ring are wave-uniform.  Columns in chunks of 64.
constexpr int kSqWaves = 4;      // rows per work-group of the fused apply (8 measured slower)
template <int CH>                // 64-column chunks per row: ceil(nb / 64)
__global__ void __launch_bounds__(64 * kSqWaves) k_modes_apply_sq(
    int32_t n, int32_t nb, const double *__restrict__ y, const double *__restrict__ yp, double *__restrict__ yo,
    const int32_t *__restrict__ nbr, const double *__restrict__ wt, const double *__restrict__ inv_s, double sigma,
    double alpha, double beta, double gam) {
    const int j = __builtin_amdgcn_readfirstlane(xcd_group(blockIdx.x, gridDim.x) * kSqWaves +
                                                 int(threadIdx.x >> 6));
    if (j >= n) return;
    const int lane = threadIdx.x & 63;
    int32_t o[3], oo[3][3];
    double w[3], ww[3][3], isk[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        o[q] = nbr[3 * j + q];
        w[q] = wt[3 * j + q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int k = o[q] >= 0 ? o[q] : j;   // a missing neighbour reads row j (not used)
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            oo[q][p] = nbr[3 * k + p];
            ww[q][p] = wt[3 * k + p];
        }
        isk[q] = inv_s[k];
    }
    const double isj = inv_s[j];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        const int c = min(lane + 64 * ch, nb - 1);
        const double yj = y[size_t(j) * nb + c];
        double yk[3], ykk[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int k = o[q] >= 0 ? o[q] : j;
            yk[q] = y[size_t(k) * nb + c];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const int l = oo[q][p];
                // row j is at hand; a missing neighbour reads row k (not used)
                ykk[q][p] = l == j ? yj : y[size_t(l >= 0 ? l : k) * nb + c];
            }
        }
        const double pv = yp ? yp[size_t(j) * nb + c] : 0.0;
        // t = (K - sigma) y at j and at the neighbours
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (o[q] >= 0) acc += w[q] * (yj - yk[q]);
        const double tj = acc * isj - sigma * yj;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (o[q] < 0) continue;
            double ak = 0.0;
#pragma unroll
            for (int p = 0; p < 3; ++p)
                if (oo[q][p] >= 0) ak += ww[q][p] * (yk[q] - ykk[q][p]);
            const double tk = ak * isk[q] - sigma * yk[q];
            s += w[q] * (tj - tk);
        }
        double out = alpha * (s * isj - sigma * tj) + beta * yj;
        if (yp) out += gam * pv;
        if (lane + 64 * ch < nb) yo[size_t(j) * nb + c] = out;
    }
}

// partial[chunk][p][q] = sum over the chunk's rows j of S_j x[j][p] z[j][q], on the FP64
// matrix cores: per step of 4 rows, v_mfma_f64_16x16x4 takes (S x)^T as the 16 x 4 operand
// (lane l: column p0 + l % 16 of row l / 16) and z as the 4 x 16 one (lane l: row l / 16,
// column q0 + l % 16), both read straight from the block (each 16 lanes read 128 contiguous
// bytes of a row).  Each wave owns a 32 x 32 block of G (2 x 2 tiles).
// grid (chunks, ceil(blocks / kGramWaves)), 64 kGramWaves work-items
constexpr int kGramWaves = 4;
constexpr int kGramUnroll = 4;      // steps of 4 rows whose loads are issued together

__global__ void __launch_bounds__(64 * kGramWaves) k_gram(int32_t n, int32_t nb, int32_t rows_per_chunk,
                                                          const double *__restrict__ x, const double *__restrict__ z,
                                                          const double *__restrict__ s, double *__restrict__ partial) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int bt = (nb + 31) / 32;
    const int blk = int(blockIdx.y) * kGramWaves + (tid >> 6);
    if (blk >= bt * bt) return;
    const int p0 = (blk / bt) * 32, q0 = (blk % bt) * 32;
    const int kr = lane >> 4, cc = lane & 15;
    const int pc[2] = {p0 + cc, p0 + 16 + cc}, qc[2] = {q0 + cc, q0 + 16 + cc};
    const int64_t r_begin = int64_t(blockIdx.x) * rows_per_chunk;
    const int64_t r_end = std::min<int64_t>(n, r_begin + rows_per_chunk);
    double4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = double4v{0.0, 0.0, 0.0, 0.0};
    for (int64_t r0 = r_begin; r0 < r_end; r0 += 4 * kGramUnroll) {
        double av[kGramUnroll][2], bv[kGramUnroll][2];
#pragma unroll
        for (int u = 0; u < kGramUnroll; ++u) {
            const int64_t row = r0 + 4 * u + kr;
            const bool in = row < r_end;
            const double sw = in ? s[row] : 0.0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                av[u][h] = in && pc[h] < nb ? sw * x[row * nb + pc[h]] : 0.0;
                bv[u][h] = in && qc[h] < nb ? z[row * nb + qc[h]] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < kGramUnroll; ++u)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][a], bv[u][b], acc[a][b], 0, 0, 0);
    }
    // the 16 x 16 result tile: lane l holds rows 4 i + l / 16, column l % 16
    double *out = partial + size_t(blockIdx.x) * nb * nb;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = p0 + 16 * a + 4 * i + kr, q = qc[b];
                if (p < nb && q < nb) out[p * nb + q] = acc[a][b][i];
            }
}

// out[k] = sum over chunks c (in order) of partial[c][k]; the loads of kSumAhead chunks are
// issued before they are added (in order)
constexpr int kSumAhead = 8;
__global__ void k_sum_chunks(int32_t chunks, int32_t len, const double *__restrict__ partial,
                             double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double acc = 0.0;
    int c = 0;
    for (; c + kSumAhead <= chunks; c += kSumAhead) {
        double v[kSumAhead];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) v[u] = partial[size_t(c + u) * len + k];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) acc += v[u];
    }
    for (; c < chunks; ++c) acc += partial[size_t(c) * len + k];
    out[k] = acc;
}

// y[j][c] = sum_k x[j][k] m[k][c]  (m upper triangular when upper != 0), or with `sub` given,
// y[j][c] = sub[j][c] - sum_k x[j][k] m[k][c] (sub may be y itself), on the FP64 matrix
// cores: v_mfma_f64_16x16x4 multiplies a 16 x 4 tile of x (lane l holds row l % 16, k l / 16)
// by a 4 x 16 tile of m (lane l holds k l / 16, column l % 16) into a 16 x 16 tile of y (lane l
// holds rows 4 i + l / 16, i < 4, column l % 16).  A work-group takes 16 kRotWaves rows (16
// per wave) and 16 kRotTiles columns; the rows of m that a step needs are staged in LDS, kRotK
// at a time, and x is read straight into the operand registers.
constexpr int kRotWaves = 4;
constexpr int kRotTiles = 2;
constexpr int kRotK = 32;

__global__ void __launch_bounds__(64 * kRotWaves) k_rotate(int32_t n, int32_t nb, const double *__restrict__ x,
                                                           const double *__restrict__ m, double *y,
                                                           int32_t upper, const double *sub) {
    constexpr int kCols = 16 * kRotTiles;
    __shared__ double ms[kRotK][kCols + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int groups = (nb + kCols - 1) / kCols;
    const int g = xcd_group(blockIdx.x, gridDim.x);
    const int64_t r0 = int64_t(g / groups) * 16 * kRotWaves;
    const int c0 = (g % groups) * kCols;
    const int64_t arow = r0 + 16 * w + (lane & 15);
    double4v acc[kRotTiles];
#pragma unroll
    for (int t = 0; t < kRotTiles; ++t) acc[t] = double4v{0.0, 0.0, 0.0, 0.0};
    // with m upper triangular, columns below c0 + kCols need rows of m below that only
    const int kend = upper ? min(nb, c0 + kCols) : nb;
    for (int k0 = 0; k0 < kend; k0 += kRotK) {
        double av[kRotK / 4];
#pragma unroll
        for (int s = 0; s < kRotK / 4; ++s) {
            const int k = k0 + 4 * s + (lane >> 4);
            av[s] = arow < n && k < nb ? x[arow * nb + k] : 0.0;
        }
        __syncthreads();                       // the previous step's rows of m are used up
        constexpr int kPer = kRotK * kCols / (64 * kRotWaves);
        double mv[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + i * 64 * kRotWaves, kk = e / kCols, cc = e % kCols;
            mv[i] = k0 + kk < nb && c0 + cc < nb ? m[(k0 + kk) * nb + c0 + cc] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = tid + i * 64 * kRotWaves;
            ms[e / kCols][e % kCols] = mv[i];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kRotK / 4; ++s)
#pragma unroll
            for (int t = 0; t < kRotTiles; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], ms[4 * s + (lane >> 4)][16 * t + (lane & 15)],
                                                               acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < kRotTiles; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + 16 * w + 4 * i + (lane >> 4);
            const int col = c0 + 16 * t + (lane & 15);
            if (row < n && col < nb) y[row * nb + col] = sub ? sub[row * nb + col] - acc[t][i] : acc[t][i];
        }
}

// One work-group: g (nb x nb, symmetric) + shift on the diagonal = R^T R; m = R^-1 (upper).
// g is overwritten.  info = 0, or k + 1 when pivot k is not positive and finite.
__global__ void __launch_bounds__(256) k_chol_inverse(int32_t nb, double *__restrict__ g, double shift,
                                                      double *__restrict__ m, int32_t *__restrict__ info) {
    __shared__ int bad;
    __shared__ double piv;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    for (int i = tid; i < nb; i += blockDim.x) g[i * nb + i] += shift;
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (tid == 0) {
            const double d = g[k * nb + k];
            if (!(d > 0.0) || !std::isfinite(d)) bad = k + 1;
            else piv = std::sqrt(d);
        }
        __syncthreads();
        if (bad) break;
        const double p = piv;
        for (int c = k + tid; c < nb; c += blockDim.x) g[k * nb + c] = c == k ? p : g[k * nb + c] / p;
        __syncthreads();
        // trailing update of the upper triangle: rows r > k, columns c >= r
        const int t = nb - k - 1;
        for (int e = tid; e < t * t; e += blockDim.x) {
            const int r = k + 1 + e / t, c = k + 1 + e % t;
            if (c >= r) g[r * nb + c] -= g[k * nb + r] * g[k * nb + c];
        }
        __syncthreads();
    }
    if (tid == 0) *info = bad;
    if (bad) return;
    // column c of R^-1 by back substitution, one thread per column
    for (int c = tid; c < nb; c += blockDim.x) {
        for (int r = nb - 1; r > c; --r) m[r * nb + c] = 0.0;
        m[c * nb + c] = 1.0 / g[c * nb + c];
        for (int r = c - 1; r >= 0; --r) {
            double acc = 0.0;
            for (int k = r + 1; k <= c; ++k) acc += g[r * nb + k] * m[k * nb + c];
            m[r * nb + c] = -acc / g[r * nb + r];
        }
    }
}

// One work-group: eigenvalues and vectors of the symmetric h (nb x nb, symmetrised first) by
// cyclic Jacobi in round-robin order (nb/2 disjoint rotations at a time).  On return theta
// holds the eigenvalues ascending and q (nb x nb, row-major) the matching eigenvectors as
// columns; h and work are overwritten.  sweeps_out: sweeps done.
__global__ void __launch_bounds__(256) k_jacobi(int32_t nb, double *__restrict__ h, double *__restrict__ work,
                                                double *__restrict__ q, double *__restrict__ theta,
                                                int32_t max_sweeps, double off_floor,
                                                int32_t *__restrict__ sweeps_out) {
    __shared__ double cs[kMaxBlock / 2 + 1], sn[kMaxBlock / 2 + 1];
    __shared__ int pp[kMaxBlock / 2 + 1], qq[kMaxBlock / 2 + 1];
    __shared__ double red[256];
    __shared__ int order[kMaxBlock];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int np = nb + (nb & 1);       // players, with a ghost when nb is odd
    const int half = np / 2;
    for (int e = tid; e < nb * nb; e += nt) {
        const int r = e / nb, c = e % nb;
        work[e] = 0.5 * (h[r * nb + c] + h[c * nb + r]);
        q[e] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += nt) h[e] = work[e];
    __syncthreads();
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // convergence: off-diagonal mass against the whole matrix
        double off = 0.0, all = 0.0;
        for (int e = tid; e < nb * nb; e += nt) {
            const double v = h[e] * h[e];
            all += v;
            if (e / nb != e % nb) off += v;
        }
        red[tid] = off;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const double off_sum = red[0];
        __syncthreads();
        red[tid] = all;
        __syncthreads();
        for (int s = nt / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        const double all_sum = red[0];
        __syncthreads();
        if (off_sum <= 1e-30 * all_sum || off_sum <= off_floor || all_sum == 0.0) break;
        for (int round = 0; round < np - 1; ++round) {
            // circle method: player 0 fixed, the others rotate
            for (int t = tid; t < half; t += nt) {
                auto player = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + round) % (np - 1); };
                const int u = player(t), v = player(np - 1 - t);
                const int a = u < v ? u : v, b = u < v ? v : u;
                double c = 1.0, s = 0.0;
                if (b < nb) {
                    const double apq = h[a * nb + b];
                    if (apq != 0.0) {
                        const double tau = (h[b * nb + b] - h[a * nb + a]) / (2.0 * apq);
                        const double tt = tau >= 0.0 ? 1.0 / (tau + std::sqrt(1.0 + tau * tau))
                                                     : -1.0 / (-tau + std::sqrt(1.0 + tau * tau));
                        c = 1.0 / std::sqrt(1.0 + tt * tt);
                        s = tt * c;
                    }
                }
                pp[t] = a;
                qq[t] = b;
                cs[t] = c;
                sn[t] = s;
            }
            __syncthreads();
            // rows: h <- J^T h
            for (int e = tid; e < half * nb; e += nt) {
                const int t = e / nb, k = e % nb;
                const int a = pp[t], b = qq[t];
                if (b >= nb || sn[t] == 0.0) continue;
                const double x = h[a * nb + k], y = h[b * nb + k];
                h[a * nb + k] = cs[t] * x - sn[t] * y;
                h[b * nb + k] = sn[t] * x + cs[t] * y;
            }
            __syncthreads();
            // columns: h <- h J, q <- q J
            for (int e = tid; e < half * nb; e += nt) {
                const int t = e / nb, k = e % nb;
                const int a = pp[t], b = qq[t];
                if (b >= nb || sn[t] == 0.0) continue;
                const double x = h[k * nb + a], y = h[k * nb + b];
                h[k * nb + a] = cs[t] * x - sn[t] * y;
                h[k * nb + b] = sn[t] * x + cs[t] * y;
                const double u = q[k * nb + a], v = q[k * nb + b];
                q[k * nb + a] = cs[t] * u - sn[t] * v;
                q[k * nb + b] = sn[t] * u + cs[t] * v;
            }
            __syncthreads();
        }
    }
    // sort ascending (rank by value, ties by index), permute the columns of q through work
    for (int i = tid; i < nb; i += nt) {
        const double v = h[i * nb + i];
        int rank = 0;
        for (int k = 0; k < nb; ++k) {
            const double u = h[k * nb + k];
            rank += (u < v) || (u == v && k < i);
        }
        order[rank] = i;
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += nt) work[e] = q[e];
    __syncthreads();
    for (int e = tid; e < nb * nb; e += nt) {
        const int r = e / nb, c = e % nb;
        q[e] = work[r * nb + order[c]];
    }
    for (int i = tid; i < nb; i += nt) theta[i] = h[order[i] * nb + order[i]];
    if (tid == 0) *sweeps_out = sweep;
}

// Packed upper triangle (row-major) of an nb x nb symmetric matrix: element (i, j), i <= j.
__device__ __forceinline__ int packed(int nb, int i, int j) { return i * (2 * nb - i - 1) / 2 + j; }

// v as held by lane src (src the same for the whole wave): two v_readlane_b32
__device__ __forceinline__ double lane_value(double v, int src) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(bits), src);
    const int hi = __builtin_amdgcn_readlane(int(bits >> 32), src);
    return __longlong_as_double((long long)(unsigned(lo)) | ((long long)(hi) << 32));
}

// for e < count: store(e, load(e)), the work-group's items in steps of kStage per work-item
// with all kStage loads issued before the first store (global memory to LDS staging)
constexpr int kStage = 8;
template <typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int count, Load load, Store store) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e0 = 0; e0 < count; e0 += kStage * nt) {
        double v[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * nt + tid;
            v[u] = e < count ? load(e) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int e = e0 + u * nt + tid;
            if (e < count) store(e, v[u]);
        }
    }
}

constexpr int kSmallThreads = 1024;   // threads of the one-work-group LDS kernels

// The Cholesky factor of g + shift I with g held in LDS (packed upper triangle, nb (nb + 1)/2
// doubles of dynamic shared memory), blocked in panels of kPanel rows: one wave factors a
// panel in registers (lane l holds columns j0 + l + 64 s), reading each pivot and multiplier
// from its lane with v_readlane, with no barrier; then all work-items apply the panel's
// rank-kPanel update to the rows below it (a group of 32 lanes per row).  g is only read; R goes to rt packed by columns
// (rt[c (c + 1)/2 + k] = R[k][c], k <= c) for k_tri_inverse.  info = 0, or 1 + the failing
// pivot's index.
constexpr int kPanel = 8;
constexpr int kTrail = kMaxBlock / 32;   // columns per lane in the trailing update
__global__ void __launch_bounds__(kSmallThreads) k_chol_lds(int32_t nb, const double *__restrict__ g, double shift,
                                                            double *__restrict__ rt, int32_t *__restrict__ info) {
    extern __shared__ double P[];
    __shared__ int bad;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
    if (tid == 0) bad = 0;
    staged_copy(
        nb * nb, [&](int e) { return g[e]; },
        [&](int e, double v) {
            const int r = e / nb, c = e % nb;
            if (c >= r) P[packed(nb, r, c)] = v + (r == c ? shift : 0.0);
        });
    __syncthreads();
    constexpr int kSlots = kMaxBlock / 64;
    for (int j0 = 0; j0 < nb; j0 += kPanel) {
        const int pw = min(kPanel, nb - j0);
        if (tid < 64) {
            double pr[kPanel][kSlots];
            // every load from a valid address (the panel's diagonal entry where the element is
            // outside the panel), so that all of them are in flight together
#pragma unroll
            for (int r = 0; r < kPanel; ++r)
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) {
                    if (j0 + 64 * sl >= nb) break;  // the same for the whole wave
                    const int c = j0 + lane + 64 * sl, rr = j0 + min(r, pw - 1);
                    const bool in = r < pw && c < nb && c >= j0 + r;
                    const double v = P[packed(nb, rr, in ? c : rr)];
                    pr[r][sl] = in ? v : 0.0;
                }
            int failed = 0;
#pragma unroll
            for (int k = 0; k < kPanel; ++k) {
                if (k >= pw || failed) continue;
                const double d = lane_value(pr[k][0], k);  // column j0 + k sits in lane k, slot 0
                if (!(d > 0.0) || !std::isfinite(d)) {
                    failed = j0 + k + 1;
                    continue;
                }
                // 1/sqrt(d): the hardware estimate and two Newton steps (each one squares the
                // relative error), a shorter dependent chain than a square root and a division
                double inv = __builtin_amdgcn_rsq(d);
#pragma unroll
                for (int it = 0; it < 2; ++it) inv = std::fma(0.5 * inv, std::fma(-d * inv, inv, 1.0), inv);
                const double piv = d * inv;
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) {
                    if (j0 + 64 * sl >= nb) break;  // the same for the whole wave
                    const int c = j0 + lane + 64 * sl;
                    if (c == j0 + k) pr[k][sl] = piv;
                    else if (c > j0 + k) pr[k][sl] *= inv;
                }
#pragma unroll
                for (int r = k + 1; r < kPanel; ++r) {
                    if (r >= pw) continue;
                    const double mult = lane_value(pr[k][0], r);  // R[j0 + k][j0 + r]
#pragma unroll
                    for (int sl = 0; sl < kSlots; ++sl) {
                        if (j0 + 64 * sl >= nb) break;  // the same for the whole wave
                        const int c = j0 + lane + 64 * sl;
                        if (c >= j0 + r && c < nb) pr[r][sl] -= mult * pr[k][sl];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < kPanel; ++r)
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) {
                    if (j0 + 64 * sl >= nb) break;  // the same for the whole wave
                    const int c = j0 + lane + 64 * sl;
                    if (r < pw && c < nb && c >= j0 + r) P[packed(nb, j0 + r, c)] = pr[r][sl];
                }
            if (failed && lane == 0) bad = failed;
        }
        __syncthreads();
        if (bad) break;
        // rows below the panel: P[r][c] -= sum over the panel rows k of R[k][r] R[k][c], a
        // group of 32 lanes per row, each lane up to kTrail columns 32 apart whose loads are
        // issued together (clamped to the row's diagonal where a column is past nb)
        for (int r0 = j0 + pw + ((tid >> 6) << 1); r0 < nb; r0 += nt >> 5) {
            const int r = r0 + ((tid >> 5) & 1);        // r0: the wave's first row
            const int ne = (nb - r0 + 31) >> 5;         // column steps of the wave's longer row
            const bool row_in = r < nb;
            const int rs = row_in ? r : r0;
            double rk[kPanel];
#pragma unroll
            for (int k = 0; k < kPanel; ++k) rk[k] = k < pw ? P[packed(nb, j0 + k, rs)] : 0.0;
            const int rowr = packed(nb, rs, 0);
            double acc[kTrail];
            int cc[kTrail];
#pragma unroll
            for (int e = 0; e < kTrail; ++e) {
                if (e >= ne) break;
                const int c = rs + (tid & 31) + 32 * e;
                cc[e] = c < nb ? c : rs;
                acc[e] = P[rowr + cc[e]];
            }
#pragma unroll
            for (int k = 0; k < kPanel; ++k) {
                if (k >= pw) break;
                const int rowk = packed(nb, j0 + k, 0);
#pragma unroll
                for (int e = 0; e < kTrail; ++e) {
                    if (e >= ne) break;
                    acc[e] -= rk[k] * P[rowk + cc[e]];
                }
            }
#pragma unroll
            for (int e = 0; e < kTrail; ++e) {
                if (e >= ne) break;
                const int c = rs + (tid & 31) + 32 * e;
                if (row_in && c < nb) P[rowr + c] = acc[e];
            }
        }
        __syncthreads();
    }
    if (tid == 0) *info = bad;
    if (bad) return;
    for (int e = tid; e < nb * nb; e += nt) {
        const int c = e / nb, k = e % nb;
        if (k <= c) rt[c * (c + 1) / 2 + k] = P[packed(nb, k, c)];
    }
}

// M = R^-1 from the column-packed R of k_chol_lds (nothing when info != 0), one wave per
// column of M: column c solves R x = e_c from the bottom, x_r = x_r / R[r][r], then
// x_k -= R[k][r] x_r for k < r, the lanes holding rows lane + 64 s.  The work-group stages the
// columns of R that its columns need, and the reciprocals of the diagonal, in LDS.  m is
// written whole (zero below the diagonal), row-major.
constexpr int kInvCols = 4;           // columns of M per work-group of k_tri_inverse

__global__ void __launch_bounds__(64 * kInvCols) k_tri_inverse(int32_t nb, const double *__restrict__ rt,
                                                               double *__restrict__ m,
                                                               const int32_t *__restrict__ info) {
    extern __shared__ double Rt[];    // packed columns 0 .. c_last, then 1 / R[r][r]
    if (*info != 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int c_last = min(nb, (int(blockIdx.x) + 1) * kInvCols) - 1;
    const int len = (c_last + 1) * (c_last + 2) / 2;
    double *dinv = Rt + len;
    staged_copy(
        len, [&](int e) { return rt[e]; }, [&](int e, double v) { Rt[e] = v; });
    __syncthreads();
    for (int r = tid; r <= c_last; r += blockDim.x) dinv[r] = 1.0 / Rt[r * (r + 1) / 2 + r];
    __syncthreads();
    const int c = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * kInvCols + (tid >> 6));
    if (c >= nb) return;
    constexpr int kSlots = kMaxBlock / 64;
    double x[kSlots];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) x[sl] = lane + 64 * sl == c ? 1.0 : 0.0;
    // column r of R (clamped to its length) and 1 / R[r][r], loaded one step ahead; slots past
    // row r hold no row that step r touches and are skipped (r is the same for the whole wave)
    auto load = [&](int r, double *colv, double &d) {
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) {
            if (sl > (r >> 6)) break;
            colv[sl] = Rt[r * (r + 1) / 2 + min(lane + 64 * sl, r)];
        }
        d = dinv[r];
    };
    double nxt[kSlots], dnxt;
    load(c, nxt, dnxt);
    for (int r = c; r >= 0; --r) {
        double cur[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) cur[sl] = nxt[sl];
        const double d = dnxt;
        if (r > 0) load(r - 1, nxt, dnxt);
        const int sr = r >> 6;
        // x_r from its lane
        double xr = x[0];
#pragma unroll
        for (int sl = 1; sl < kSlots; ++sl)
            if (sl == sr) xr = x[sl];
        const double mr = lane_value(xr, r & 63) * d;
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) {
            if (sl > sr) break;
            const int k = lane + 64 * sl;
            const double upd = x[sl] - cur[sl] * mr;
            x[sl] = k < r ? upd : (k == r ? mr : x[sl]);
        }
    }
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
        const int k = lane + 64 * sl;
        if (k < nb) m[size_t(k) * nb + c] = k <= c ? x[sl] : 0.0;
    }
}

// Cyclic Jacobi on the symmetric h held in LDS (packed upper triangle of np x np, np = nb
// rounded up to even, the padding row and column zero), np/2 disjoint rotations per round in
// round-robin order: position 0 stays, every other player moves down one position per round,
// and pair slot t joins positions t and np - 1 - t.  Every 2 x 2 block of h that two pairs
// s <= t share becomes J_s^T B J_t.  The blocks are dealt to the work-items once (kJacobiItems
// at most each, the same (s, t) slots every round; the pairs in a slot change), and a
// work-item issues the loads of a group of its blocks before it computes any.
// The next round's pairs are known in advance (slot t' joins the players now at positions
// t' + 1 and np - t', or 0 and 1 for t' = 0), and the off-diagonal entry of each lies in one
// block of the current round: the work-item updating that block also computes the next
// round's rotation for it, the two diagonal entries re-derived from the current pairs'
// entries as their own diagonal blocks derive them.  A round is then one barrier; only a
// sweep's first round (after the convergence test) computes its rotations in a phase of its
// own.  The rotations are written to rot[sweep][round][pair] = (c, s) for k_jacobi_vectors; on
// return theta holds the eigenvalues ascending, order[i] the diagonal position of the i-th,
// and sweeps_out the sweeps done.
constexpr int kJacobiItems = 5;     // blocks per work-item: (96 x 95 / 2 - 96) / (1024 - 128), rounded up
constexpr int kJacobiGroup = 3;     // blocks whose loads are issued together
constexpr int kJacobiNp = 192;      // largest np held in LDS
constexpr int kJacobiHalf = kJacobiNp / 2;
constexpr int kJacobiLds = kJacobiNp * (kJacobiNp + 1) / 2;

__device__ __forceinline__ int row_offset(int np, int i) { return i * (2 * np - i - 1) / 2; }

// a pair's entries h[a][a], h[b][b], h[a][b] before its rotation
struct PairEntries {
    double x, y, z;
};

// the rotation that annihilates h[a][b]; skipped (identity) below rounding of the diagonal
__device__ __forceinline__ bool jacobi_angle(double app, double aqq, double apq, double &c, double &sn) {
    c = 1.0;
    sn = 0.0;
    if (!(std::fabs(apq) > 1e-16 * (std::fabs(app) + std::fabs(aqq)))) return false;
    const double tau = (aqq - app) / (2.0 * apq);
    const double tt = tau >= 0.0 ? 1.0 / (tau + std::sqrt(1.0 + tau * tau)) : -1.0 / (-tau + std::sqrt(1.0 + tau * tau));
    c = 1.0 / std::sqrt(1.0 + tt * tt);
    sn = tt * c;
    return true;
}

// J^T B J of a 2 x 2 block between pairs with rotations (c1, s1) (rows) and (c2, s2) (columns)
__device__ __forceinline__ void rotate_block(double c1, double s1, double c2, double s2, double h00, double h01,
                                             double h10, double h11, double &y00, double &y01, double &y10,
                                             double &y11) {
    // J_s^T B: rows mix; then (J_s^T B) J_t: columns mix
    const double x00 = std::fma(c1, h00, -s1 * h10), x01 = std::fma(c1, h01, -s1 * h11);
    const double x10 = std::fma(s1, h00, c1 * h10), x11 = std::fma(s1, h01, c1 * h11);
    y00 = std::fma(c2, x00, -s2 * x01);
    y01 = std::fma(s2, x00, c2 * x01);
    y10 = std::fma(c2, x10, -s2 * x11);
    y11 = std::fma(s2, x10, c2 * x11);
}

__global__ void __launch_bounds__(kSmallThreads) k_jacobi_lds(int32_t nb, const double *__restrict__ h,
                                                              double2 *__restrict__ rot, double *__restrict__ theta,
                                                              int32_t *__restrict__ order_out, int32_t max_sweeps,
                                                              double off_floor, int32_t *__restrict__ sweeps_out) {
    __shared__ double P[kJacobiLds];  // static, so that its address folds into the LDS offsets
    __shared__ int4 pr[2][kJacobiHalf];            // pair: 8 a, 8 b, 8 x row offsets (a < b)
    __shared__ double2 cs[2][kJacobiHalf];          // pair rotation (c, s)
    __shared__ PairEntries pe[2][kJacobiHalf];
    __shared__ unsigned char lowa[2][kJacobiHalf];  // 1: a holds the slot's low position
    __shared__ double red[kSmallThreads / 64][2];
    __shared__ int order[kJacobiNp];
    __shared__ int rotated;            // a rotation was applied in the current sweep
    const int tid = threadIdx.x, nt = blockDim.x;
    const int np = nb + (nb & 1), half = np / 2;
    // with fewer than 3 pairs two of the next round's pairs can share a block: those sizes
    // compute every round's rotations in a phase of their own
    const bool merged = half >= 3;
    if (tid == 0) rotated = 0;
    // h symmetrised; entries of h below the diagonal are read in the transposed order
    staged_copy(
        nb * nb, [&](int e) { return h[e]; },
        [&](int e, double v) {
            const int r = e / nb, c = e % nb;
            if (c >= r) P[row_offset(np, r) + c] = r == c ? v : 0.5 * v;
        });
    __syncthreads();
    staged_copy(
        nb * nb, [&](int e) { return h[(e % nb) * nb + e / nb]; },
        [&](int e, double v) {
            const int r = e / nb, c = e % nb;
            if (c > r) P[row_offset(np, r) + c] += 0.5 * v;
        });
    if (np > nb)
        for (int r = tid; r < np; r += nt) P[row_offset(np, r) + nb] = 0.0;
    // Work split.  The first t0 work-items (whole waves) own the pair slots t < half: the
    // diagonal block (t, t) and, when merged, the block that holds next-round pair t's
    // off-diagonal entry, for which they also compute the next rotation.  The other
    // work-items take the remaining blocks (s, t), s < t, in row-major order, at most
    // kJacobiItems each, the same slots every round.
    const int t0 = (half + 63) / 64 * 64;
    // the block (row r, column c) holding next pair tn's entry, and where its players sit:
    // bit 0 (1): the row (column) slot gives its high-position player, bit 2: the row slot's
    // player takes the next pair's low position
    auto next_block = [&](int tn, int &r, int &c) {
        if (tn == 0) {
            r = 0;
            c = 1;
            return 4;                                  // low of 0 (next low), low of 1
        }
        if (tn <= half - 2) {
            r = tn - 1;
            c = tn + 1;
            return 1;                                  // high of tn - 1, low of tn + 1 (next low)
        }
        r = half - 2;
        c = half - 1;
        return 3;                                      // high of both, the column's next low
    };
    auto designated = [&](int r, int c) {
        return merged && ((r == 0 && c == 1) || (c == r + 2 && r + 1 <= half - 2) || (r == half - 2 && c == half - 1));
    };
    int item[kJacobiItems];
    int n_items = 0;                                   // the most any work-item has (the same for all)
    {
        const int rest = half * (half - 1) / 2 - (merged ? half : 0);
        const int workers = nt - t0;
        n_items = (rest + workers - 1) / workers;
#pragma unroll
        for (int i = 0; i < kJacobiItems; ++i) {
            item[i] = -1;
            const int m = tid - t0 + i * workers;
            if (tid < t0 || m >= rest) continue;
            // row r holds half - 1 - r blocks, less the designated ones
            int r = 0, before = 0;
            for (;; ++r) {
                // (a row's designated blocks sit in its first two columns)
                int cnt = half - 1 - r;
                for (int c = r + 1; c < half && c <= r + 2; ++c) cnt -= designated(r, c);
                if (m < before + cnt) break;
                before += cnt;
            }
            int j = m - before, c = r + 1;
            for (;; ++c)
                if (!designated(r, c) && j-- == 0) break;
            item[i] = (r << 16) | c;
        }
    }
    auto player = [&](int k, int round) {
        if (k == 0) return 0;
        const int z = k - 1 + round;
        return 1 + (z >= np - 1 ? z - (np - 1) : z);
    };
    // the rotations of one round in a phase of their own, into table buffer bf
    auto rotations = [&](int sweep, int round, int bf) {
        for (int t = tid; t < half; t += nt) {
            const int u = player(t, round), v = player(np - 1 - t, round);
            const int a = u < v ? u : v, b = u < v ? v : u;
            const int oa = row_offset(np, a), ob = row_offset(np, b);
            const double app = P[oa + a], aqq = P[ob + b], apq = P[oa + b];
            double c = 1.0, sn = 0.0;
            if (b < nb && jacobi_angle(app, aqq, apq, c, sn)) rotated = 1;
            pr[bf][t] = make_int4(8 * a, 8 * b, 8 * oa, 8 * ob);
            cs[bf][t] = make_double2(c, sn);
            pe[bf][t] = PairEntries{app, aqq, apq};
            lowa[bf][t] = u < v;
            rot[(size_t(sweep) * (np - 1) + round) * half + t] = make_double2(c, sn);
        }
    };
    __syncthreads();
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // off-diagonal mass against the whole matrix (wave sums, then one thread)
        double off = 0.0, all = 0.0;
        for (int e = tid; e < nb * nb; e += nt) {
            const int r = e / nb, c = e % nb;
            if (c < r) continue;
            const double v = P[row_offset(np, r) + c];
            all += (r == c ? 1.0 : 2.0) * v * v;
            if (r != c) off += 2.0 * v * v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            all += __shfl_xor(all, o);
        }
        if ((tid & 63) == 0) {
            red[tid >> 6][0] = off;
            red[tid >> 6][1] = all;
        }
        __syncthreads();
        double off_sum = 0.0, all_sum = 0.0;
        for (int w = 0; w < nt / 64; ++w) {
            off_sum += red[w][0];
            all_sum += red[w][1];
        }
        const bool none_last = sweep > 0 && !rotated;
        __syncthreads();
        if (off_sum <= 1e-30 * all_sum || off_sum <= off_floor || all_sum == 0.0 || none_last) break;
        if (tid == 0) rotated = 0;
        __syncthreads();
        rotations(sweep, 0, 0);
        __syncthreads();
        for (int round = 0; round < np - 1; ++round) {
            const int cb = round & 1, nbf = cb ^ 1;
            const bool ahead = merged && round + 1 < np - 1;   // this round computes the next one's rotations
            // packed position of (i, j) from the row offsets
            // (byte offsets: the table holds 8 x the indices and row offsets)
            auto at = [](int i, int oi, int j, int oj) { return i <= j ? oi + j : oj + i; };
            auto el = [&](int off) -> double & { return *reinterpret_cast<double *>(reinterpret_cast<char *>(P) + off); };
            if (tid < t0) {
                if (tid < half) {
                    const int t = tid;
                    // the pair's diagonal block: (a, b) is annihilated by its own rotation
                    const int4 p = pr[cb][t];
                    const double2 q = cs[cb][t];
                    const int iaa = p.z + p.x, iab = p.z + p.y, ibb = p.w + p.y;
                    const double haa = el(iaa), hab = el(iab), hbb = el(ibb);
                    double y00, y01, y10, y11;
                    rotate_block(q.x, q.y, q.x, q.y, haa, hab, hab, hbb, y00, y01, y10, y11);
                    el(iaa) = y00;
                    el(ibb) = y11;
                    el(iab) = q.y != 0.0 ? 0.0 : y01;
                    if (merged) {
                        int s1i, s2i;
                        const int bits = next_block(t, s1i, s2i);
                        const int4 p1 = pr[cb][s1i], p2 = pr[cb][s2i];
                        const double2 q1 = cs[cb][s1i], q2 = cs[cb][s2i];
                        const int i00 = at(p1.x, p1.z, p2.x, p2.z), i01 = at(p1.x, p1.z, p2.y, p2.w);
                        const int i10 = at(p1.y, p1.w, p2.x, p2.z), i11 = at(p1.y, p1.w, p2.y, p2.w);
                        rotate_block(q1.x, q1.y, q2.x, q2.y, el(i00), el(i01), el(i10), el(i11), y00, y01, y10, y11);
                        el(i00) = y00;
                        el(i01) = y01;
                        el(i10) = y10;
                        el(i11) = y11;
                        if (ahead) {
                            // member index (0: a, 1: b) of the row and column slots' players
                            const int ir = bool(bits & 1) == bool(lowa[cb][s1i]) ? 1 : 0;
                            const int ic = bool(bits & 2) == bool(lowa[cb][s2i]) ? 1 : 0;
                            const double offd = ir ? (ic ? y11 : y10) : (ic ? y01 : y00);
                            const int id_r = (ir ? p1.y : p1.x) >> 3, id_c = (ic ? p2.y : p2.x) >> 3;
                            // new diagonal entries, as the pairs' own diagonal blocks compute them
                            auto diag = [&](const double2 &qq, const PairEntries &e, int im) {
                                double d00, d01, d10, d11;
                                rotate_block(qq.x, qq.y, qq.x, qq.y, e.x, e.z, e.z, e.y, d00, d01, d10, d11);
                                return im ? d11 : d00;
                            };
                            const double dr = diag(q1, pe[cb][s1i], ir), dc = diag(q2, pe[cb][s2i], ic);
                            const bool r_first = id_r < id_c;
                            const int a = r_first ? id_r : id_c, b = r_first ? id_c : id_r;
                            const double app = r_first ? dr : dc, aqq = r_first ? dc : dr;
                            double c = 1.0, sn = 0.0;
                            if (b < nb && jacobi_angle(app, aqq, offd, c, sn)) rotated = 1;
                            const int oa = row_offset(np, a), ob = row_offset(np, b);
                            pr[nbf][t] = make_int4(8 * a, 8 * b, 8 * oa, 8 * ob);
                            cs[nbf][t] = make_double2(c, sn);
                            pe[nbf][t] = PairEntries{app, aqq, offd};
                            const int low_id = (bits & 4) ? id_r : id_c;
                            lowa[nbf][t] = low_id == a;
                            rot[(size_t(sweep) * (np - 1) + round + 1) * half + t] = make_double2(c, sn);
                        }
                    }
                }
            } else {
                // the remaining blocks in groups of kJacobiGroup: all loads of a group, then
                // its updates
#pragma unroll
                for (int g = 0; g < kJacobiItems; g += kJacobiGroup) {
                    if (g >= n_items) break;             // the same for the whole work-group
                    int idx[kJacobiGroup][4];
                    double hv[kJacobiGroup][4];
#pragma unroll
                    for (int j = 0; j < kJacobiGroup; ++j) {
                        const int i = g + j;
                        if (i >= kJacobiItems || i >= n_items) break;
                        const int code = item[i] < 0 ? 1 : item[i];   // (0, 1) is a valid block
                        const int4 p1 = pr[cb][code >> 16], p2 = pr[cb][code & 0xffff];
                        idx[j][0] = at(p1.x, p1.z, p2.x, p2.z);
                        idx[j][1] = at(p1.x, p1.z, p2.y, p2.w);
                        idx[j][2] = at(p1.y, p1.w, p2.x, p2.z);
                        idx[j][3] = at(p1.y, p1.w, p2.y, p2.w);
#pragma unroll
                        for (int q = 0; q < 4; ++q) hv[j][q] = el(idx[j][q]);
                    }
#pragma unroll
                    for (int j = 0; j < kJacobiGroup; ++j) {
                        const int i = g + j;
                        if (i >= kJacobiItems || i >= n_items) break;
                        if (item[i] < 0) continue;
                        const double2 q1 = cs[cb][item[i] >> 16], q2 = cs[cb][item[i] & 0xffff];
                        double y00, y01, y10, y11;
                        rotate_block(q1.x, q1.y, q2.x, q2.y, hv[j][0], hv[j][1], hv[j][2], hv[j][3], y00, y01, y10,
                                     y11);
                        el(idx[j][0]) = y00;
                        el(idx[j][1]) = y01;
                        el(idx[j][2]) = y10;
                        el(idx[j][3]) = y11;
                    }
                }
            }
            __syncthreads();
            if (!merged && round + 1 < np - 1) {
                rotations(sweep, round + 1, nbf);
                __syncthreads();
            }
        }
    }
    for (int i = tid; i < nb; i += nt) {
        const double v = P[row_offset(np, i) + i];
        int rank = 0;
        for (int k = 0; k < nb; ++k) {
            const double u = P[row_offset(np, k) + k];
            rank += (u < v) || (u == v && k < i);
        }
        order[rank] = i;
    }
    __syncthreads();
    for (int i = tid; i < nb; i += nt) {
        theta[i] = P[row_offset(np, order[i]) + order[i]];
        order_out[i] = order[i];
    }
    if (tid == 0) *sweeps_out = sweep;
}

// Eigenvectors from the rotation log of k_jacobi_lds: row k of Q starts as e_k and takes
// every round's rotations of its entries, Q <- Q J; the columns are then put in the order of
// the sorted eigenvalues.  A work-group takes kVecRows rows (work-item t applies pair t's
// rotation to each), and keeps the log entries of the next kVecAhead rounds in flight while it
// applies the current one.  blockDim >= nb/2.
constexpr int kVecRows = 4;
constexpr int kVecAhead = 4;

__global__ void k_jacobi_vectors(int32_t nb, const double2 *__restrict__ rot, const int32_t *__restrict__ sweeps,
                                 const int32_t *__restrict__ order, double *__restrict__ q) {
    __shared__ double row[kVecRows][kMaxBlock + 1];
    const int k0 = blockIdx.x * kVecRows, tid = threadIdx.x;
    const int np = nb + (nb & 1), half = np / 2;
    for (int i = tid; i < kVecRows * np; i += blockDim.x) {
        const int rr = i / np, c = i % np;
        row[rr][c] = c == k0 + rr ? 1.0 : 0.0;
    }
    __syncthreads();
    const int total = *sweeps * (np - 1);     // rounds in the log
    const bool active = tid < half;
    double2 ring[kVecAhead];
#pragma unroll
    for (int j = 0; j < kVecAhead; ++j)
        ring[j] = active && j < total ? rot[size_t(j) * half + tid] : make_double2(1.0, 0.0);
    int round = 0;
    for (int base = 0; base < total; base += kVecAhead) {
#pragma unroll
        for (int j = 0; j < kVecAhead; ++j) {
            const int idx = base + j;
            if (idx >= total) break;                 // the same for the whole work-group
            const double2 r = ring[j];
            if (active && idx + kVecAhead < total) ring[j] = rot[size_t(idx + kVecAhead) * half + tid];
            if (active && r.y != 0.0) {
                auto player = [&](int kk) {
                    if (kk == 0) return 0;
                    const int z = kk - 1 + round;
                    return 1 + (z >= np - 1 ? z - (np - 1) : z);
                };
                const int u = player(tid), v = player(np - 1 - tid);
                const int a = u < v ? u : v, b = u < v ? v : u;
                if (b < nb)
#pragma unroll
                    for (int rr = 0; rr < kVecRows; ++rr) {
                        const double x = row[rr][a], y = row[rr][b];
                        row[rr][a] = r.x * x - r.y * y;
                        row[rr][b] = r.y * x + r.x * y;
                    }
            }
            round = round + 1 == np - 1 ? 0 : round + 1;
            __syncthreads();
        }
    }
    for (int i = tid; i < kVecRows * nb; i += blockDim.x) {
        const int rr = i / nb, c = i % nb;
        if (k0 + rr < nb) q[(k0 + rr) * nb + c] = row[rr][order[c]];
    }
}

// partial[chunk][c] = sum over the chunk's rows of S_j (kv[j][c] - theta_c v[j][c])^2
__global__ void k_residual(int32_t n, int32_t nb, int32_t rows_per_chunk, const double *__restrict__ v,
                           const double *__restrict__ kv, const double *__restrict__ theta,
                           const double *__restrict__ s, double *__restrict__ partial) {
    const int c = threadIdx.x;
    if (c >= nb) return;
    const int64_t r_begin = int64_t(blockIdx.x) * rows_per_chunk;
    const int64_t r_end = std::min<int64_t>(n, r_begin + rows_per_chunk);
    const double th = theta[c];
    double acc = 0.0;
    int64_t j = r_begin;
    // kSumAhead rows' loads in flight, accumulated in row order
    for (; j + kSumAhead <= r_end; j += kSumAhead) {
        double a[kSumAhead], b[kSumAhead], w[kSumAhead];
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            a[u] = kv[(j + u) * nb + c];
            b[u] = v[(j + u) * nb + c];
            w[u] = s[j + u];
        }
#pragma unroll
        for (int u = 0; u < kSumAhead; ++u) {
            const double r = a[u] - th * b[u];
            acc += w[u] * r * r;
        }
    }
    for (; j < r_end; ++j) {
        const double r = kv[j * nb + c] - th * v[j * nb + c];
        acc += s[j] * r * r;
    }
    partial[size_t(blockIdx.x) * nb + c] = acc;
}

// x[j][c] = 2 u - 1 with u = (splitmix64(seed + j nb + c) >> 11) 2^-53 (canonical j), for the
// columns c with flags[c] != 0 (every column when flags is null; the others are left as they are)
__global__ void k_random_block(int32_t n, int32_t nb, const int32_t *__restrict__ canon, uint64_t seed,
                               double *__restrict__ x, const int32_t *__restrict__ flags) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= uint32_t(n) * uint32_t(nb)) return;
    const uint32_t j = g / uint32_t(nb), c = g - j * uint32_t(nb);
    if (flags && !flags[c]) return;
    uint64_t z = seed + uint64_t(canon[j]) * uint64_t(nb) + c + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[g] = 2.0 * (double(z >> 11) * 0x1.0p-53) - 1.0;
}

// x[j][c] = 0 for the columns with flags[c] == 0
__global__ void k_keep_columns(int32_t n, int32_t nb, const int32_t *__restrict__ flags, double *__restrict__ x) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= uint32_t(n) * uint32_t(nb)) return;
    if (!flags[g % uint32_t(nb)]) x[g] = 0.0;
}

// out[i][canon[j]] = x[j][cols[i]] for i < count: block columns transposed into canonical
// triangle order.  A work-group moves a 64-row x 16-column tile through LDS (reads along the
// row, writes along the triangles).
constexpr int kExportRows = 64, kExportCols = 16;
__global__ void __launch_bounds__(256) k_export_columns(int32_t n, int32_t nb, const double *__restrict__ x,
                                                        const int32_t *__restrict__ canon,
                                                        const int32_t *__restrict__ cols, int32_t count,
                                                        double *__restrict__ out) {
    __shared__ double tile[kExportCols][kExportRows + 1];
    const int tid = threadIdx.x;
    const int64_t j0 = int64_t(blockIdx.x) * kExportRows;
    const int i0 = int(blockIdx.y) * kExportCols;
    for (int e = tid; e < kExportRows * kExportCols; e += blockDim.x) {
        const int r = e / kExportCols, c = e % kExportCols;
        const int64_t j = j0 + r;
        tile[c][r] = j < n && i0 + c < count ? x[j * nb + cols[i0 + c]] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < kExportRows * kExportCols; e += blockDim.x) {
        const int c = e / kExportRows, r = e % kExportRows;
        const int64_t j = j0 + r;
        const int i = i0 + c;
        if (j < n && i < count) out[int64_t(i) * n + canon[j]] = tile[c][r];
    }
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct ModeSolver {
    int32_t n = 0, nb = 0, chunks = 0, rows_per_chunk = 0;
    // highest modes: the solver works on K' = top - K, whose lowest modes are K's highest
    bool reversed = false;
    double top = 0.0;
    size_t packed_bytes = 0;           // LDS for a packed nb x nb triangle, 0 = does not fit
    hipStream_t st = nullptr;
    DeviceBuffer arena;                // one allocation that the buffers below are views of
    DeviceBuffer nbr, wt, inv_s, s, canon;
    DeviceBuffer buf[5];               // block-sized buffers
    DeviceBuffer xb[4];                // further block-sized buffers (the spectrum's locked windows)
    DeviceBuffer g, m, h, q, work, theta, partial, small_i, rot, order;
    DeviceBuffer cols;                 // 3 nb int32: a column list and two column flag arrays

    double *B(int i) const { return buf[i].as<double>(); }

    // `extra` (<= 4) further block-sized buffers in xb
    int alloc(const Mesh &mesh, const double *gamma, int32_t nblock, double *upper, int extra = 0) {
        n = int32_t(mesh.nt);
        nb = nblock;
        const int64_t nt = mesh.nt;
        std::vector<int32_t> slot(nt), hn(3 * nt, -1), hc(nt);
        std::vector<double> hw(3 * nt, 0.0), hinv(nt), hs(nt);
        for (int64_t k = 0; k < nt; ++k) slot[mesh.perm_t[k]] = int32_t(k);
        double bound = 0.0;
        for (int64_t k = 0; k < nt; ++k) {
            const int32_t j = mesh.perm_t[k];
            hc[k] = j;
            hs[k] = mesh.S[j];
            hinv[k] = 1.0 / mesh.S[j];
            double row = 0.0;
            for (int qd = 0; qd < 3; ++qd) {
                const int32_t i = mesh.A[3 * j + qd];
                if (!mesh.interior(i)) continue;
                const double gm = gamma ? gamma[i] : 1.0;
                const double w = gm * gm * mesh.elen[i] / mesh.d[i];
                const int32_t o = mesh.R[i] == j ? mesh.L[i] : mesh.R[i];
                hn[3 * k + qd] = slot[o];
                hw[3 * k + qd] = w;
                // Gershgorin row of S^(1/2) K S^(-1/2): diagonal plus off-diagonal magnitudes
                row += w / mesh.S[j] + w / std::sqrt(mesh.S[j] * mesh.S[o]);
            }
            bound = std::max(bound, row);
        }
        *upper = bound;
        const size_t blk = size_t(nt) * nb * sizeof(double);
        rows_per_chunk = int32_t(std::max<int64_t>(128, (nt + 511) / 512));
        chunks = int32_t((nt + rows_per_chunk - 1) / rows_per_chunk);
        const size_t sq = size_t(nb) * nb * sizeof(double);
        const int np = nb + (nb & 1);
        // every device buffer is a 256-byte aligned view of one allocation
        std::vector<std::pair<DeviceBuffer *, size_t>> parts = {
            {&buf[0], blk}, {&buf[1], blk}, {&buf[2], blk}, {&buf[3], blk}, {&buf[4], blk},
            {&nbr, hn.size() * 4}, {&wt, hw.size() * 8}, {&inv_s, size_t(nt) * 8}, {&s, size_t(nt) * 8},
            {&canon, size_t(nt) * 4}, {&g, sq}, {&m, sq}, {&h, sq}, {&q, sq}, {&work, sq},
            {&theta, size_t(nb) * 8}, {&partial, size_t(chunks) * nb * nb * sizeof(double)},
            {&small_i, 2 * sizeof(int32_t)},
            {&rot, size_t(kJacobiSweeps) * (np - 1) * (np / 2) * sizeof(double2)},
            {&order, size_t(nb) * sizeof(int32_t)}, {&cols, size_t(3) * nb * sizeof(int32_t)}};
        for (int i = 0; i < std::min(extra, 4); ++i) parts.push_back({&xb[i], blk});
        auto aligned = [](size_t b) { return (b + 255) / 256 * 256; };
        size_t total = 0;
        for (const auto &pt : parts) total += aligned(pt.second);
        int rc = arena.alloc(total);
        if (rc) return rc;
        size_t off = 0;
        for (const auto &pt : parts) {
            pt.first->p = static_cast<char *>(arena.p) + off;
            pt.first->bytes = pt.second;
            pt.first->owned = false;
            off += aligned(pt.second);
        }
        int device = 0, lds_limit = 65536;
        TYEE_HIP(hipGetDevice(&device));
        TYEE_HIP(hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, device));
        // the small kernels also hold up to about 7 KB of static shared memory
        // (np: the Jacobi kernel pads an odd nb by one row and column)
        const size_t tri_bytes = size_t(np) * (np + 1) / 2 * sizeof(double);
        // (the Jacobi kernel's remaining blocks must fit the work-items beyond the pair slots)
        const int jh = np / 2, jt0 = (jh + 63) / 64 * 64;
        const int jrest = jh * (jh - 1) / 2 - (jh >= 3 ? jh : 0);
        packed_bytes = tri_bytes + 8 * 1024 <= size_t(lds_limit) && jrest <= kJacobiItems * (kSmallThreads - jt0) &&
                               np * (np + 1) / 2 <= kJacobiLds
                           ? tri_bytes
                           : 0;
        TYEE_HIP(hipMemcpyAsync(nbr.p, hn.data(), hn.size() * 4, hipMemcpyHostToDevice, st));
        TYEE_HIP(hipMemcpyAsync(wt.p, hw.data(), hw.size() * 8, hipMemcpyHostToDevice, st));
        TYEE_HIP(hipMemcpyAsync(inv_s.p, hinv.data(), nt * 8, hipMemcpyHostToDevice, st));
        TYEE_HIP(hipMemcpyAsync(s.p, hs.data(), nt * 8, hipMemcpyHostToDevice, st));
        TYEE_HIP(hipMemcpyAsync(canon.p, hc.data(), nt * 4, hipMemcpyHostToDevice, st));
        TYEE_HIP(hipStreamSynchronize(st));
        return TYEE_OK;
    }

    unsigned grid_items() const { return unsigned((int64_t(n) * nb + kBlock - 1) / kBlock); }

    int apply(const double *y, const double *yp, double *yo, double alpha, double beta, double gam) {
        if (reversed) {  // alpha (top - K) y + beta y = -alpha K y + (beta + alpha top) y
            beta += alpha * top;
            alpha = -alpha;
        }
        const dim3 grid((n + kApplyWaves - 1) / kApplyWaves), threads(64 * kApplyWaves);
        const int32_t *nb_ = nbr.as<int32_t>();
        const double *wt_ = wt.as<double>(), *is_ = inv_s.as<double>();
        if (nb % 2 == 0 && nb <= 256) {
            switch ((nb + 127) / 128) {
            case 1: hipLaunchKernelGGL(k_modes_apply2<1>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, alpha, beta, gam); break;
            default: hipLaunchKernelGGL(k_modes_apply2<2>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, alpha, beta, gam); break;
            }
            TYEE_HIP(hipGetLastError());
            return TYEE_OK;
        }
        switch ((nb + 63) / 64) {
        case 1: hipLaunchKernelGGL(k_modes_apply<1>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, alpha, beta, gam); break;
        case 2: hipLaunchKernelGGL(k_modes_apply<2>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, alpha, beta, gam); break;
        case 3: hipLaunchKernelGGL(k_modes_apply<3>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, alpha, beta, gam); break;
        default: hipLaunchKernelGGL(k_modes_apply<4>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, alpha, beta, gam); break;
        }
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    // yo = alpha (K - sigma)^2 y + beta y + gam yp, one launch
    int apply_sq(const double *y, const double *yp, double *yo, double sigma, double alpha, double beta, double gam) {
        const dim3 grid((n + kSqWaves - 1) / kSqWaves), threads(64 * kSqWaves);
        const int32_t *nb_ = nbr.as<int32_t>();
        const double *wt_ = wt.as<double>(), *is_ = inv_s.as<double>();
        switch ((nb + 63) / 64) {
        case 1: hipLaunchKernelGGL(k_modes_apply_sq<1>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, sigma, alpha, beta, gam); break;
        case 2: hipLaunchKernelGGL(k_modes_apply_sq<2>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, sigma, alpha, beta, gam); break;
        case 3: hipLaunchKernelGGL(k_modes_apply_sq<3>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, sigma, alpha, beta, gam); break;
        default: hipLaunchKernelGGL(k_modes_apply_sq<4>, grid, threads, 0, st, n, nb, y, yp, yo, nb_, wt_, is_, sigma, alpha, beta, gam); break;
        }
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    // out (nb x nb) = x^T S z
    int gram(const double *x, const double *z, double *out) {
        const int bt = (nb + 31) / 32;
        hipLaunchKernelGGL(k_gram, dim3(chunks, (bt * bt + kGramWaves - 1) / kGramWaves), dim3(64 * kGramWaves), 0, st,
                           n, nb, rows_per_chunk, x, z, s.as<double>(), partial.as<double>());
        TYEE_HIP(hipGetLastError());
        const int len = nb * nb;
        hipLaunchKernelGGL(k_sum_chunks, dim3((len + 255) / 256), dim3(256), 0, st, chunks, len,
                           partial.as<double>(), out);
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    int rotate(const double *x, const double *mat, double *y, bool upper, const double *sub = nullptr) {
        const int rows = 16 * kRotWaves, cols = 16 * kRotTiles;
        hipLaunchKernelGGL(k_rotate, dim3(((n + rows - 1) / rows) * ((nb + cols - 1) / cols)), dim3(64 * kRotWaves), 0,
                           st, n, nb, x, mat, y, int32_t(upper), sub);
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    // One Cholesky QR pass: src -> dst (src is left intact when the factorisation fails).
    // *ok = false when a pivot is not positive.
    // With `ahead`, the rotation into dst is launched before the status is read (dst then holds
    // garbage on failure, so dst must not be a block that a failure needs).
    int cholqr_pass(int src, int dst, bool shifted, bool *ok, bool ahead = false) {
        int rc = gram(B(src), B(src), g.as<double>());
        if (rc) return rc;
        double shift = 0.0;
        if (shifted) {
            // shift = 11 (n nb + nb (nb + 1)) u ||G||_2, ||G||_2 bounded by the trace
            std::vector<double> hg(size_t(nb) * nb);
            TYEE_HIP(hipMemcpyAsync(hg.data(), g.p, hg.size() * 8, hipMemcpyDeviceToHost, st));
            TYEE_HIP(hipStreamSynchronize(st));
            double tr = 0.0;
            for (int i = 0; i < nb; ++i) tr += hg[size_t(i) * nb + i];
            shift = 11.0 * (double(n) * nb + double(nb) * (nb + 1)) * 0x1.0p-53 * tr;
        }
        if (packed_bytes) {
            hipLaunchKernelGGL(k_chol_lds, dim3(1), dim3(kSmallThreads), packed_bytes, st, nb, g.as<double>(), shift,
                               work.as<double>(), small_i.as<int32_t>());
            TYEE_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_tri_inverse, dim3((nb + kInvCols - 1) / kInvCols), dim3(64 * kInvCols),
                               (size_t(nb) * (nb + 1) / 2 + nb) * sizeof(double), st, nb, work.as<double>(),
                               m.as<double>(), small_i.as<int32_t>());
        } else
            hipLaunchKernelGGL(k_chol_inverse, dim3(1), dim3(256), 0, st, nb, g.as<double>(), shift,
                               m.as<double>(), small_i.as<int32_t>());
        TYEE_HIP(hipGetLastError());
        int32_t info = 0;
        TYEE_HIP(hipMemcpyAsync(&info, small_i.p, 4, hipMemcpyDeviceToHost, st));
        if (ahead) {
            const int rc = rotate(B(src), m.as<double>(), B(dst), true);
            if (rc) return rc;
        }
        TYEE_HIP(hipStreamSynchronize(st));
        *ok = info == 0;
        return *ok && !ahead ? rotate(B(src), m.as<double>(), B(dst), true) : TYEE_OK;
    }

    // The block in buffer ix made S-orthonormal, using buffer iy as well; *out names the
    // buffer that holds the result.  Cholesky QR twice, which suffices while the block's
    // condition number stays below about u^(-1/2) (the filter degree is capped for that);
    // if a factorisation fails, the shifted Cholesky QR three times (Fukaya et al., SIAM J.
    // Sci. Comput. 2020) from the same block.  TYEE_EUNSTABLE when that fails too.
    // With `once`, a single Cholesky QR: the block comes out well conditioned (orthonormal to
    // about u cond^2), which is all a following filter pass needs.
    // With `shifted`, the shifted Cholesky QR three times straight away: for a block filtered
    // with a growth beyond what Cholesky QR twice can take (condition numbers up to about u^-1).
    int orthonormalise(int ix, int iy, int *out, bool once = false, bool shifted = false) {
        bool ok = false;
        int rc = TYEE_OK;
        if (shifted) {
            rc = cholqr_pass(ix, iy, true, &ok);
            if (!rc && ok) rc = cholqr_pass(iy, ix, false, &ok);
            if (!rc && ok) rc = cholqr_pass(ix, iy, false, &ok);
            if (rc) return rc;
            if (!ok) return fail(TYEE_EUNSTABLE, "mode block lost rank");
            *out = iy;
            return TYEE_OK;
        }
        rc = cholqr_pass(ix, iy, false, &ok, true);   // iy is scratch if this pass fails
        if (!rc && ok && once) {
            *out = iy;
            return TYEE_OK;
        }
        if (!rc && ok) rc = cholqr_pass(iy, ix, false, &ok);
        if (rc) return rc;
        if (ok) {
            *out = ix;
            return TYEE_OK;
        }
        // ix still holds the block when either pass failed (the first pass writes only iy, and
        // the second writes ix only on success)
        rc = cholqr_pass(ix, iy, true, &ok);
        if (!rc && ok) rc = cholqr_pass(iy, ix, false, &ok);
        if (!rc && ok) rc = cholqr_pass(ix, iy, false, &ok);
        if (rc) return rc;
        if (!ok) return fail(TYEE_EUNSTABLE, "mode block lost rank");
        *out = iy;
        return TYEE_OK;
    }

    // The lowest buffer index not in `used`.
    static int pick(std::initializer_list<int> used) {
        for (int i = 0; i < 5; ++i)
            if (std::find(used.begin(), used.end(), i) == used.end()) return i;
        return -1;
    }

    // Rayleigh-Ritz of the S-orthonormal block in buffer iv (scratch iz): Ritz vectors to
    // buffer ov, K times them to buffer okv (four distinct buffers), Ritz values to host.
    // off_floor: the Jacobi also stops once the off-diagonal sum of squares is below it
    int rayleigh_ritz(int iv, int iz, int ov, int okv, std::vector<double> &ritz, int max_sweeps, double off_floor) {
        int rc = apply(B(iv), nullptr, B(iz), 1.0, 0.0, 0.0);
        if (!rc) rc = gram(B(iv), B(iz), h.as<double>());
        if (rc) return rc;
        if (packed_bytes) {
            hipLaunchKernelGGL(k_jacobi_lds, dim3(1), dim3(kSmallThreads), 0, st, nb, h.as<double>(),
                               rot.as<double2>(), theta.as<double>(), order.as<int32_t>(), max_sweeps, off_floor,
                               small_i.as<int32_t>() + 1);
            TYEE_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_jacobi_vectors, dim3((nb + kVecRows - 1) / kVecRows), dim3(128), 0, st, nb,
                               rot.as<double2>(),
                               small_i.as<int32_t>() + 1, order.as<int32_t>(), q.as<double>());
        } else {
            hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), 0, st, nb, h.as<double>(), work.as<double>(),
                               q.as<double>(), theta.as<double>(), max_sweeps, off_floor, small_i.as<int32_t>() + 1);
        }
        TYEE_HIP(hipGetLastError());
        rc = rotate(B(iv), q.as<double>(), B(ov), false);
        if (!rc) rc = rotate(B(iz), q.as<double>(), B(okv), false);
        if (rc) return rc;
        ritz.resize(nb);
        TYEE_HIP(hipMemcpyAsync(ritz.data(), theta.p, size_t(nb) * 8, hipMemcpyDeviceToHost, st));
        TYEE_HIP(hipStreamSynchronize(st));
        return TYEE_OK;
    }

    int residuals(int iv, int ikv, std::vector<double> &res) {
        hipLaunchKernelGGL(k_residual, dim3(chunks), dim3(((nb + 63) / 64) * 64), 0, st, n, nb, rows_per_chunk,
                           B(iv), B(ikv), theta.as<double>(), s.as<double>(), partial.as<double>());
        TYEE_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_sum_chunks, dim3((nb + 255) / 256), dim3(256), 0, st, chunks, nb, partial.as<double>(),
                           g.as<double>());
        TYEE_HIP(hipGetLastError());
        res.resize(nb);
        TYEE_HIP(hipMemcpyAsync(res.data(), g.p, size_t(nb) * 8, hipMemcpyDeviceToHost, st));
        TYEE_HIP(hipStreamSynchronize(st));
        for (double &r : res) r = std::sqrt(std::max(r, 0.0));
        return TYEE_OK;
    }

    // Deflation in metric (7): x <- x - V (V^T S x) for each locked block V in xb (S-orthonormal
    // columns, the unused ones zero), in place in buffer ix.
    int project(int ix, const std::vector<int> &locked) {
        for (int l : locked) {
            int rc = gram(xb[l].as<double>(), B(ix), g.as<double>());
            if (!rc) rc = rotate(xb[l].as<double>(), g.as<double>(), B(ix), false, B(ix));
            if (rc) return rc;
        }
        return TYEE_OK;
    }

    // The filter below run on (K - sigma)^2, whose spectrum lies in [0, mu_max] and whose lowest
    // modes are the modes of K nearest sigma: degree-k Chebyshev damping of [a, mu_max] with
    // growth measured from mu = 0, each step one launch of the fused (K - sigma)^2 apply.  Reads
    // buffer `in`, rotates through three others; the result lands in buffer *out.
    int filter_sq(int in, int degree, double a, double mu_max, double sigma, int *out) {
        const double e = 0.5 * (mu_max - a), c = 0.5 * (mu_max + a);
        const double sigma1 = -e / c;
        double sg = sigma1;
        const int w0 = pick({in}), w1 = pick({in, w0}), w2 = pick({in, w0, w1});
        // y1 = (sigma1 / e) ((K - sigma)^2 - c) y0
        int rc = apply_sq(B(in), nullptr, B(w0), sigma, sigma1 / e, -sigma1 * c / e, 0.0);
        if (rc) return rc;
        int prev = in, cur = w0;
        for (int k = 2; k <= degree; ++k) {
            const double sn = 1.0 / (2.0 / sigma1 - sg);
            const int nxt = (w0 != cur && w0 != prev) ? w0 : (w1 != cur && w1 != prev) ? w1 : w2;
            // y_k = (2 sn / e) ((K - sigma)^2 - c) y_{k-1} - sg sn y_{k-2}
            rc = apply_sq(B(cur), B(prev), B(nxt), sigma, 2.0 * sn / e, -2.0 * sn * c / e, -sg * sn);
            if (rc) return rc;
            prev = cur;
            cur = nxt;
            sg = sn;
        }
        *out = cur;
        return TYEE_OK;
    }

    // Degree-k filter of the block in buffer `in` damping [a, b_up] with a0 the estimate of
    // the lowest eigenvalue; it rotates through three other buffers (`in` is only read) and
    // the result lands in buffer *out.
    int filter(int in, int degree, double a, double b_up, double a0, int *out) {
        const double e = 0.5 * (b_up - a), c = 0.5 * (b_up + a);
        const double sigma1 = e / (a0 - c);
        double sigma = sigma1;
        const int w0 = pick({in}), w1 = pick({in, w0}), w2 = pick({in, w0, w1});
        // y1 = (sigma1 / e) (K - c) y0
        int rc = apply(B(in), nullptr, B(w0), sigma1 / e, -sigma1 * c / e, 0.0);
        if (rc) return rc;
        int prev = in, cur = w0;
        for (int k = 2; k <= degree; ++k) {
            const double sigma_new = 1.0 / (2.0 / sigma1 - sigma);
            const int nxt = (w0 != cur && w0 != prev) ? w0 : (w1 != cur && w1 != prev) ? w1 : w2;
            // y_{k} = (2 sigma_new / e)(K - c) y_{k-1} - sigma sigma_new y_{k-2}
            rc = apply(B(cur), B(prev), B(nxt), 2.0 * sigma_new / e, -2.0 * sigma_new * c / e, -sigma * sigma_new);
            if (rc) return rc;
            prev = cur;
            cur = nxt;
            sigma = sigma_new;
        }
        *out = cur;
        return TYEE_OK;
    }
};

}  // namespace
}  // namespace tyee

extern "C" int tyee_mesh_modes(const tyee_mesh *mesh, const double *gamma, int32_t which, int64_t n_modes,
                               int32_t block, int32_t degree, double tol, int32_t max_iter, uint64_t seed,
                               void *stream, double *omega2, double *modes, double *residual,
                               tyee_modes_stats *stats) {
    using namespace tyee;
    if (!mesh || !omega2) return fail(TYEE_EINVAL, "null argument");
    if (which != TYEE_MODES_LOWEST && which != TYEE_MODES_HIGHEST)
        return fail(TYEE_EINVAL, "which must be TYEE_MODES_LOWEST or TYEE_MODES_HIGHEST");
    const Mesh &msh = mesh->m;
    const int64_t nt = msh.nt;
    if (n_modes < 1 || n_modes > std::min<int64_t>(nt, kMaxBlock))
        return fail(TYEE_EINVAL, "n_modes must be in 1 .. min(n_triangles, 256)");
    int64_t nb = block;
    if (nb == 0) nb = std::min<int64_t>({nt, int64_t(kMaxBlock), n_modes + std::max<int64_t>(16, n_modes / 4)});
    if (nb < std::max<int64_t>(n_modes, 2) || nb > std::min<int64_t>(nt, kMaxBlock))
        return fail(TYEE_EINVAL, "block must be in max(n_modes, 2) .. min(n_triangles, 256)");
    if (nt * nb >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "n_triangles x block must be below 2^31");
    if (degree == 0) degree = 128;
    if (degree < 1 || degree > 100000) return fail(TYEE_EINVAL, "degree must be in 1 .. 100000");
    if (!(tol > 0.0) || max_iter < 1) return fail(TYEE_EINVAL, "tol > 0 and max_iter >= 1 required");
    const auto t_start = std::chrono::steady_clock::now();
    try {
        ModeSolver sv;
        sv.st = static_cast<hipStream_t>(stream);
        EventPair ev;
        TYEE_HIP(hipEventCreate(&ev.a));
        TYEE_HIP(hipEventCreate(&ev.b));
        double filter_ms = 0.0;
        int64_t applies = 0;
        double b_up = 0.0;
        int rc = sv.alloc(msh, gamma, int32_t(nb), &b_up);
        if (rc) return rc;
        if (!(b_up > 0.0)) return fail(TYEE_EINVAL, "mesh has no interior edge");
        sv.reversed = which == TYEE_MODES_HIGHEST;
        sv.top = b_up;  // top - K has its spectrum in [0, b_up] too
        // random start, S-orthonormalised, then a first Rayleigh-Ritz for the bounds
        hipLaunchKernelGGL(k_random_block, dim3(sv.grid_items()), dim3(kBlock), 0, sv.st, sv.n, sv.nb,
                           sv.canon.as<int32_t>(), seed, sv.B(0), nullptr);
        TYEE_HIP(hipGetLastError());
        int ob = 1;
        // a tall random block is well conditioned: one Cholesky QR leaves it orthonormal to
        // rounding
        rc = sv.orthonormalise(0, 1, &ob, 4 * nb <= nt);
        std::vector<double> ritz, res;
        int vb = ModeSolver::pick({ob, 2}), kvb = ModeSolver::pick({ob, 2, vb});  // Ritz vectors, K times them
        // a random block smaller than the space is never converged: a few Jacobi sweeps give
        // Ritz values close enough for the first filter's bounds
        // off-diagonal entries of H move Ritz pairs by about their size: below 1e-3 of the
        // residual tolerance they no longer matter
        const double off_floor = (1e-3 * tol * b_up) * (1e-3 * tol * b_up);
        if (!rc) rc = sv.rayleigh_ritz(ob, 2, vb, kvb, ritz, nb < nt ? kStartSweeps : kJacobiSweeps, off_floor);
        if (!rc) rc = sv.residuals(vb, kvb, res);
        applies += 1;
        auto converged = [&]() {
            for (int64_t c = 0; c < n_modes; ++c)
                if (!(res[c] <= tol * b_up)) return false;
            return true;
        };
        int32_t it = 0;
        bool done = !rc && converged();
        while (!rc && !done && it < max_iter) {
            const double a = ritz[nb - 1], a0 = std::min(ritz[0], a);
            // a block that spans the whole space is exact after Rayleigh-Ritz: no filter
            const bool filtered = nb < nt && a < b_up * (1.0 - 1e-12) && a0 < a;
            // cap the degree so that the lowest mode grows at most 1e7 times more than the modes
            // at the cut: the filtered block then keeps a condition number that Cholesky QR twice
            // handles
            const double x0 = (0.5 * (b_up + a) - a0) / (0.5 * (b_up - a));
            int deg = degree;
            if (x0 > 1.0) deg = int(std::max(1.0, std::min(double(degree), std::floor(std::log(2e7) / std::acosh(x0)))));
            // kFilterPasses filter passes, each followed by Cholesky QR, per Rayleigh-Ritz step:
            // subspace iteration needs no Rayleigh-Ritz between passes
            int in = vb;
            for (int pass = 0; pass < (filtered ? kFilterPasses : 1) && !rc; ++pass) {
                int fo = in;
                if (filtered) {
                    TYEE_HIP(hipEventRecord(ev.a, sv.st));
                    rc = sv.filter(in, deg, a, b_up, a0, &fo);
                    TYEE_HIP(hipEventRecord(ev.b, sv.st));
                    applies += deg;
                }
                // a pass that another filter pass follows needs a well-conditioned block only
                const bool last = pass + 1 == (filtered ? kFilterPasses : 1);
                if (!rc) rc = sv.orthonormalise(fo, ModeSolver::pick({fo}), &in, !last);
                if (!rc && filtered) {
                    float ms = 0.0f;
                    TYEE_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                    filter_ms += ms;
                }
            }
            if (rc) break;
            const int spare = ModeSolver::pick({in});
            vb = ModeSolver::pick({in, spare});
            kvb = ModeSolver::pick({in, spare, vb});
            // far from convergence the Rayleigh-Ritz step only has to give the filter its bounds
            // and an orthonormal basis of the same subspace (any rotation of it will do): a few
            // Jacobi sweeps suffice.  Once the previous step's residuals are within kNearTol of
            // the tolerance, the Jacobi runs to its end.
            double worst = 0.0;
            for (int64_t c = 0; c < n_modes; ++c) worst = std::max(worst, res[c]);
            const int sweeps = worst <= kNearTol * tol * b_up ? kJacobiSweeps : kMidSweeps;
            rc = sv.rayleigh_ritz(in, spare, vb, kvb, ritz, sweeps, off_floor);
            if (!rc) rc = sv.residuals(vb, kvb, res);
            if (rc) break;
            applies += 1;                          // the Rayleigh-Ritz product K V
            ++it;
            done = converged();
        }
        if (rc) return rc;
        for (int64_t c = 0; c < n_modes; ++c) omega2[c] = sv.reversed ? b_up - ritz[c] : ritz[c];
        if (residual)
            for (int64_t c = 0; c < n_modes; ++c) residual[c] = res.empty() ? 1.0 : res[c] / b_up;
        if (stats) {
            stats->iters = it;
            stats->applies = applies;
            stats->lambda_bound = b_up;
            stats->filter_ms = filter_ms;
            stats->total_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        }
        if (modes) {
            std::vector<double> hv(size_t(nt) * nb);
            TYEE_HIP(hipMemcpyAsync(hv.data(), sv.B(vb), hv.size() * 8, hipMemcpyDeviceToHost, sv.st));
            TYEE_HIP(hipStreamSynchronize(sv.st));
            for (int64_t k = 0; k < nt; ++k) {
                const int32_t j = msh.perm_t[k];
                for (int64_t c = 0; c < n_modes; ++c) modes[c * nt + j] = hv[size_t(k) * nb + c];
            }
        }
        return done ? TYEE_OK : fail(TYEE_ENOTCONVERGED, "mode residuals above tol after max_iter iterations");
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}


namespace tyee {
namespace {

constexpr int64_t kSpectrumBlock = 192;   // default block of the whole-spectrum solver
constexpr int kLocked = 3;                // windows kept for deflation (xb[0..2]; xb[3] stages exports)

// Rows row0.. of the host matrix modes[n_t][n_t] (canonical triangle order) from the block
// columns listed first in sv.cols (count of them, in that order), through xb[3].
int export_modes(ModeSolver &sv, int vb, int64_t count, double *modes, int64_t row0) {
    if (!modes || count <= 0) return TYEE_OK;
    const dim3 grid((sv.n + kExportRows - 1) / kExportRows, unsigned((count + kExportCols - 1) / kExportCols));
    hipLaunchKernelGGL(k_export_columns, grid, dim3(256), 0, sv.st, sv.n, sv.nb, sv.B(vb), sv.canon.as<int32_t>(),
                       sv.cols.as<int32_t>(), int32_t(count), sv.xb[3].as<double>());
    TYEE_HIP(hipGetLastError());
    TYEE_HIP(hipMemcpyAsync(modes + row0 * sv.n, sv.xb[3].p, size_t(count) * sv.n * sizeof(double),
                            hipMemcpyDeviceToHost, sv.st));
    TYEE_HIP(hipStreamSynchronize(sv.st));
    return TYEE_OK;
}

bool spectrum_trace() {
    static const bool on = std::getenv("TYEE_SPECTRUM_TRACE") != nullptr;
    return on;
}

}  // namespace
}  // namespace tyee

extern "C" int tyee_mesh_spectrum(const tyee_mesh *mesh, const double *gamma, int32_t block, int32_t degree,
                                  double tol, int32_t max_iter, uint64_t seed, void *stream, double *omega2,
                                  double *modes, double *residual, tyee_spectrum_stats *stats) {
    using namespace tyee;
    if (!mesh || !omega2) return fail(TYEE_EINVAL, "null argument");
    const Mesh &msh = mesh->m;
    const int64_t nt = msh.nt;
    int64_t nb = block;
    if (nb == 0) nb = std::min<int64_t>(nt, kSpectrumBlock);
    if (nb < std::min<int64_t>(nt, 16) || nb > std::min<int64_t>(nt, kMaxBlock))
        return fail(TYEE_EINVAL, "block must be in min(n_triangles, 16) .. min(n_triangles, 256)");
    if (nt * nb >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "n_triangles x block must be below 2^31");
    if (degree == 0) degree = 100000;
    if (degree < 2 || degree > 100000) return fail(TYEE_EINVAL, "degree must be in 2 .. 100000");
    if (!(tol > 0.0) || max_iter < 1) return fail(TYEE_EINVAL, "tol > 0 and max_iter >= 1 required");
    const auto t_start = std::chrono::steady_clock::now();
    tyee_spectrum_stats st{};
    auto finish = [&](int rc) {
        st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        if (stats) *stats = st;
        return rc;
    };
    try {
        ModeSolver sv;
        sv.st = static_cast<hipStream_t>(stream);
        EventPair ev;
        TYEE_HIP(hipEventCreate(&ev.a));
        TYEE_HIP(hipEventCreate(&ev.b));
        double b_up = 0.0;
        int rc = sv.alloc(msh, gamma, int32_t(nb), &b_up, modes ? kLocked + 1 : kLocked);
        if (rc) return rc;
        if (!(b_up > 0.0)) return fail(TYEE_EINVAL, "mesh has no interior edge");
        st.lambda_bound = b_up;
        sv.top = b_up;  // lambda_bound - K has its spectrum in [0, b_up] too
        const double res_tol = tol * b_up;
        const double off_floor = (1e-3 * res_tol) * (1e-3 * res_tol);
        std::vector<double> ritz, res;
        // host copy of sv.cols: the accepted columns in output order, the columns to keep in the
        // locked copy, the columns to restart at random in the next window
        std::vector<int32_t> hcols(size_t(3) * nb, 0);
        auto upload_cols = [&]() -> int {
            TYEE_HIP(hipMemcpyAsync(sv.cols.p, hcols.data(), hcols.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                    sv.st));
            TYEE_HIP(hipStreamSynchronize(sv.st));
            return TYEE_OK;
        };
        auto accept_outputs = [&](const std::vector<int64_t> &acc, const std::vector<double> &val, int64_t row0,
                                  int vb) -> int {
            for (size_t i = 0; i < acc.size(); ++i) {
                omega2[row0 + int64_t(i)] = val[i];
                st.max_residual = std::max(st.max_residual, res[acc[i]] / b_up);
                if (residual) residual[row0 + int64_t(i)] = res[acc[i]] / b_up;
                hcols[i] = int32_t(acc[i]);
            }
            int rc2 = upload_cols();
            if (!rc2) rc2 = export_modes(sv, vb, int64_t(acc.size()), modes, row0);
            return rc2;
        };

        if (nb == nt) {
            // the block spans the whole space: one Rayleigh-Ritz step is exact
            hipLaunchKernelGGL(k_random_block, dim3(sv.grid_items()), dim3(kBlock), 0, sv.st, sv.n, sv.nb,
                               sv.canon.as<int32_t>(), seed, sv.B(0), nullptr);
            TYEE_HIP(hipGetLastError());
            int ob = 0;
            rc = sv.orthonormalise(0, 1, &ob);
            const int spare = ModeSolver::pick({ob}), vb = ModeSolver::pick({ob, spare}),
                      kvb = ModeSolver::pick({ob, spare, vb});
            if (!rc) rc = sv.rayleigh_ritz(ob, spare, vb, kvb, ritz, kJacobiSweeps, off_floor);
            if (!rc) rc = sv.residuals(vb, kvb, res);
            if (rc) return finish(rc);
            std::vector<int64_t> acc(nt);
            for (int64_t c = 0; c < nt; ++c) acc[c] = c;
            rc = accept_outputs(acc, ritz, 0, vb);
            if (rc) return finish(rc);
            st.windows = 1;
            st.applies = 1;
            st.found = nt;
            for (int64_t c = 0; c < nt; ++c)
                if (!(res[c] <= res_tol)) return finish(fail(TYEE_ENOTCONVERGED, "mode residuals above tol"));
            return finish(TYEE_OK);
        }

        // Spectrum slicing.  Window 0 takes the top modes with the low-pass filter of
        // lambda_bound - K (which also gives lambda_max, the top of the spectrum the other
        // filters have to damp); window 1 the lowest modes with the low-pass filter of K; each
        // further window filters with (K - sigma)^2, beta being the boundary below which every
        // mode is found, and runs up to the top window's boundary.  A window's start block is
        // S-orthogonalised against the modes of the last windows (deflation in metric (7), as the
        // paper withdraws the found eigenvectors from the initial vector), and the filter passes
        // then run without projections: a projection in every pass would hold the block exactly
        // orthogonal to modes that are themselves only accurate to the tolerance, and that error
        // would pass on from window to window.  Found modes that grow back are recognised outside
        // the window and set aside.  sigma sits a quarter of the block's reach R above beta
        // (R^2 = the largest mu of the block, below), so that the ball of radius R about sigma
        // reaches down past beta; sigma moves down when the reach shrinks (the spectrum gets
        // denser).
        //
        // Which Ritz pairs a window may accept: the filter favours the block's directions by
        // mu = ||(K - z) v||^2 = res^2 + (theta - z)^2 (z = sigma, or the bottom of the filtered
        // operator's spectrum), so every mode with a smaller mu than a converged Ritz vector is
        // in the block and converged before it.  The trusted set is the block's converged Ritz
        // pairs taken in order of mu up to the first one that has not converged, and it holds
        // every mode with (lambda - z)^2 below that one's mu; unconverged vectors (mixtures from
        // both sides of sigma) may have Ritz values anywhere and are passed over.  A window is
        // accepted once that ball reaches down to beta, with its boundary in the widest gap
        // among the trusted Ritz values, so that each eigenvalue is accepted exactly once.
        enum { kLinear, kSquared, kTop };
        const int64_t target = (2 * nb + 4) / 5;     // trusted pairs a window waits for
        const double gap_min = 16.0 * res_tol;      // a boundary gap the Ritz errors cannot cross
        constexpr double kSigmaAt = 0.25, kSigmaMax = 0.35;   // sigma - beta in units of the reach
        constexpr double kSqGrowth = 1e10;                     // filter growth per interior pass
        int64_t low = 0, high = 0;                  // pairs found from the bottom, from the top
        double beta = -HUGE_VAL, beta_top = HUGE_VAL;   // the window runs over [beta, beta_top)
        double lam_hi = b_up;                       // the top of the spectrum (lambda_max once known)
        double sigma = 0.0, a_hint = 0.0, min_gap = HUGE_VAL;
        std::vector<int> locked;                    // xb indices of the windows deflated against
        int next_slot = 0;
        int vb = -1, kvb = -1;                      // Ritz vectors of the last window, K times them
        std::vector<double> mu(nb);
        std::vector<int64_t> by_mu(nb);
        // The block's reach in mu, for the filter's pass band [0, a]: its largest mu.  After a
        // pass whose band held fewer modes than the block has vectors, the spare vectors come
        // out of the orthonormalisation as unfiltered noise with a huge mu; they do not measure
        // the reach: the band is then widened in the ratio of all vectors to the filtered ones
        // (at a constant density of modes, their count grows with the radius sqrt(a)).
        auto reach_of = [&](const std::vector<double> &m, double a_used) {
            double top = 0.0, top_kept = 0.0;
            int64_t spare = 0;
            for (double v : m) {
                top = std::max(top, v);
                if (a_used > 0.0 && v > 4.0 * a_used) ++spare;
                else top_kept = std::max(top_kept, v);
            }
            if (spare == 0 || spare == nb) return top;
            const double grow = double(nb) / double(nb - spare);
            return std::min(top, top_kept * grow * grow);
        };
        for (int32_t win = 0; low + high < nt; ++win) {
            const int64_t remaining = nt - low - high;
            const int mode = win == 0 ? kTop : win == 1 ? kLinear : kSquared;
            sv.reversed = mode == kTop;
            // start: the last window's block with its accepted and stale columns restarted at
            // random (the window after the top one starts afresh)
            const bool warm_start = vb >= 0 && mode == kSquared;
            int x0 = 0;
            if (warm_start) {
                x0 = ModeSolver::pick({vb});
                TYEE_HIP(hipMemcpyAsync(sv.B(x0), sv.B(vb), size_t(nt) * nb * sizeof(double),
                                        hipMemcpyDeviceToDevice, sv.st));
            }
            const uint64_t wseed = seed + uint64_t(win) * uint64_t(nt) * uint64_t(nb);
            hipLaunchKernelGGL(k_random_block, dim3(sv.grid_items()), dim3(kBlock), 0, sv.st, sv.n, sv.nb,
                               sv.canon.as<int32_t>(), wseed, sv.B(x0),
                               warm_start ? sv.cols.as<int32_t>() + 2 * nb : nullptr);
            TYEE_HIP(hipGetLastError());
            rc = sv.project(x0, locked);
            int ob = x0;
            if (!rc) rc = sv.orthonormalise(x0, ModeSolver::pick({x0}), &ob);
            if (rc == TYEE_EUNSTABLE && warm_start) {
                // the kept columns were too close to the deflated modes: all columns at random
                hipLaunchKernelGGL(k_random_block, dim3(sv.grid_items()), dim3(kBlock), 0, sv.st, sv.n, sv.nb,
                                   sv.canon.as<int32_t>(), wseed, sv.B(x0), nullptr);
                TYEE_HIP(hipGetLastError());
                rc = sv.project(x0, locked);
                if (!rc) rc = sv.orthonormalise(x0, ModeSolver::pick({x0}), &ob);
            }
            int spare = ModeSolver::pick({ob});
            vb = ModeSolver::pick({ob, spare});
            kvb = ModeSolver::pick({ob, spare, vb});
            if (!rc) rc = sv.rayleigh_ritz(ob, spare, vb, kvb, ritz, kStartSweeps, off_floor);
            if (!rc) rc = sv.residuals(vb, kvb, res);
            if (rc) return finish(rc);
            st.applies += 1;
            auto lam_of = [&](int64_t c) { return mode == kTop ? b_up - ritz[c] : ritz[c]; };
            std::vector<int64_t> acc, aside, warm;  // accepted (ascending), found before, kept
            double new_bound = 0.0;                 // the window's new boundary
            int64_t prev_good = -1;
            int stalled = 0;                       // iterations without more trusted pairs
            double a_used = 0.0;                   // the pass band of the last filter pass
            for (int32_t it = 0;; ++it) {
                const bool last_try = it >= max_iter;
                // trusted set: converged pairs in order of mu up to the first unconverged one
                for (int64_t c = 0; c < nb; ++c) {
                    const double z = mode == kSquared ? ritz[c] - sigma : ritz[c];
                    mu[c] = res[c] * res[c] + z * z;
                    by_mu[c] = c;
                }
                std::stable_sort(by_mu.begin(), by_mu.end(), [&](int64_t x, int64_t y) { return mu[x] < mu[y]; });
                std::vector<int64_t> good;          // trusted and inside [beta, beta_top)
                aside.clear();
                int64_t trusted = 0;
                for (; trusted < nb && res[by_mu[trusted]] <= res_tol; ++trusted) {
                    const int64_t c = by_mu[trusted];
                    const double lam = lam_of(c);
                    if (lam >= beta && lam < beta_top) good.push_back(c);
                    else aside.push_back(c);
                }
                // the trusted ball holds every mode with (lambda - sigma)^2 below mu_stop
                const double mu_stop = trusted < nb ? mu[by_mu[trusted]] : HUGE_VAL;
                const bool covers = mode != kSquared || (sigma - beta) * (sigma - beta) < mu_stop;
                std::sort(good.begin(), good.end(), [&](int64_t x, int64_t y) { return lam_of(x) < lam_of(y); });
                const int64_t g = int64_t(good.size());
                // a window whose trusted pairs no longer grow in number (its ball cannot grow: a
                // sparse part of the spectrum, the rest of the block outside the window) settles
                // for what it has
                stalled = covers && g >= 2 && g <= prev_good + 1 ? stalled + 1 : 0;
                prev_good = g;
                const bool settle = last_try || trusted == nb || stalled >= 1;
                bool done = false;
                if (covers && g == remaining) {
                    acc = good;                     // every mode left: no boundary needed
                    warm.clear();
                    done = true;
                } else if (covers && g > remaining) {
                    return finish(fail(TYEE_EUNSTABLE, "more converged modes in the window than remain"));
                } else if (covers && g >= 2 && (g >= target + 1 || settle)) {
                    // take all but the last of them (from the window's own end: the bottom for
                    // the top window), cut in the widest gap of the far fifth, else anywhere
                    const int64_t want = g - 1;
                    double best = -1.0;
                    int64_t cut = -1;               // boundary between good[cut] and good[cut + 1]
                    for (int pass = 0; pass < 2 && best < gap_min; ++pass) {
                        int64_t k0 = 0, k1 = want;
                        if (pass == 0) {
                            if (mode == kTop) k1 = std::max<int64_t>(1, want / 5);
                            else k0 = (4 * want) / 5;
                        }
                        for (int64_t k = k0; k < k1; ++k) {
                            const double gap = lam_of(good[k + 1]) - lam_of(good[k]);
                            if (gap > best) {
                                best = gap;
                                cut = k;
                            }
                        }
                    }
                    if (best >= gap_min) {
                        new_bound = 0.5 * (lam_of(good[cut]) + lam_of(good[cut + 1]));
                        if (mode == kTop) {
                            acc.assign(good.begin() + cut + 1, good.end());
                            warm.clear();
                        } else {
                            acc.assign(good.begin(), good.begin() + cut + 1);
                            warm.assign(good.begin() + cut + 1, good.end());
                        }
                        min_gap = std::min(min_gap, best / b_up);
                        done = true;
                    }
                }
                if (spectrum_trace()) {
                    std::fprintf(stderr,
                                 "[spectrum] win %d mode %d it %d beta %.9g sigma %.9g trusted %lld good %lld aside %zu "
                                 "covers %d%s |",
                                 win, mode, it, beta, sigma, (long long)trusted, (long long)g, aside.size(),
                                 int(covers), done ? " accept" : "");
                    for (int64_t k = 0; k < std::min<int64_t>(nb, 4); ++k)
                        std::fprintf(stderr, " (%.4g %.1e)", lam_of(by_mu[k]) - (mode == kSquared ? sigma : 0.0),
                                     res[by_mu[k]] / b_up);
                    std::fprintf(stderr, "\n");
                }
                if (done) {
                    st.iters += it;
                    st.below += int64_t(aside.size());
                    break;
                }
                if (last_try) {
                    st.iters += it;
                    return finish(fail(TYEE_ENOTCONVERGED, "a spectral window did not converge within max_iter"));
                }
                // a filter pass, the orthonormalisation, Rayleigh-Ritz
                bool filtered = false;
                int deg = 1;
                double a = 0.0, a0 = 0.0, mu_max = 0.0, upper = 0.0;
                if (mode == kSquared) {
                    a = reach_of(mu, a_used);
                    if (it == 0 && a_hint > 0.0) a = std::min(a, a_hint);
                    // keep sigma within reach of beta
                    if (sigma - beta > kSigmaMax * std::sqrt(a)) {
                        const double moved = beta + kSigmaAt * std::sqrt(a);
                        for (int64_t c = 0; c < nb; ++c) {   // the block's mu about the new sigma
                            const double z = ritz[c] - moved;
                            mu[c] = res[c] * res[c] + z * z;
                        }
                        sigma = moved;
                        a = reach_of(mu, a_used);
                        if (it == 0 && a_hint > 0.0) a = std::min(a, a_hint);
                    }
                    a_used = a;
                    mu_max = std::max(sigma, lam_hi - sigma);
                    mu_max *= mu_max;
                    filtered = a > 0.0 && a < mu_max * (1.0 - 1e-12);
                    if (filtered) {
                        // growth from mu = 0 to the cut at most kSqGrowth: one pass then converges
                        // the modes near sigma (the block is orthonormalised by the shifted
                        // Cholesky QR, which takes such condition numbers)
                        const double x0m = (mu_max + a) / (mu_max - a);
                        deg = int(std::max(1.0, std::min(double(degree / 2), std::floor(std::log(kSqGrowth) / std::acosh(x0m)))));
                    }
                } else {
                    // the growth is capped from the bottom of the filtered operator's spectrum
                    // (K, and lambda_bound - K, are non-negative), below which no mode lies; the
                    // damped interval ends at the top of that spectrum
                    upper = mode == kTop ? b_up : lam_hi;
                    a = ritz[nb - 1];
                    a0 = 0.0;
                    filtered = a < upper * (1.0 - 1e-12) && a0 < a;
                    const double x0 = (0.5 * (upper + a) - a0) / (0.5 * (upper - a));
                    deg = degree;
                    if (filtered && x0 > 1.0)
                        deg = int(std::max(1.0, std::min(double(degree), std::floor(std::log(2e7) / std::acosh(x0)))));
                }
                if (spectrum_trace())
                    std::fprintf(stderr, "[spectrum]   filter a %g mu_max %g deg %d\n", a, mu_max, deg);
                // interior windows: one pass per Rayleigh-Ritz step, which costs little beside a
                // pass at these degrees and lets the window stop as soon as it has converged
                const int passes = !filtered ? 1 : mode == kSquared ? 1 : kFilterPasses;
                int in = vb;
                for (int pass = 0; pass < passes && !rc; ++pass) {
                    const bool last = pass + 1 == passes;
                    auto run_pass = [&](int d, bool high_growth) -> int {
                        int fo = in;
                        if (filtered) {
                            TYEE_HIP(hipEventRecord(ev.a, sv.st));
                            int rc2;
                            if (mode == kSquared) {
                                rc2 = sv.filter_sq(in, d, a, mu_max, sigma, &fo);
                                st.applies += 2 * d;
                                st.sq_launches += d;
                            } else {
                                rc2 = sv.filter(in, d, a, upper, a0, &fo);
                                st.applies += d;
                            }
                            TYEE_HIP(hipEventRecord(ev.b, sv.st));
                            if (rc2) return rc2;
                        }
                        // the scratch buffer spares `in`, so that a failed pass can be redone
                        int out = in;
                        const int rc2 = sv.orthonormalise(fo, ModeSolver::pick({fo, in}), &out, !last, high_growth);
                        if (filtered) {   // the orthonormalisation has waited for the stream
                            TYEE_HIP(hipEventSynchronize(ev.b));
                            float ms = 0.0f;
                            TYEE_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                            st.filter_ms += ms;
                            if (mode == kSquared) st.sq_ms += ms;
                        }
                        if (!rc2) in = out;
                        return rc2;
                    };
                    const bool high_growth = mode == kSquared && filtered;
                    rc = run_pass(deg, high_growth);
                    if (rc == TYEE_EUNSTABLE && high_growth) {
                        // the block was worse conditioned than the shifted Cholesky QR takes:
                        // the pass again at the growth that Cholesky QR twice handles
                        ++st.retries;
                        if (spectrum_trace()) std::fprintf(stderr, "[spectrum]   pass redone at low growth\n");
                        const double x0m = (mu_max + a) / (mu_max - a);
                        const int safe = int(std::max(1.0, std::min(double(deg), std::floor(std::log(2e7) / std::acosh(x0m)))));
                        rc = run_pass(safe, false);
                    }
                }
                if (rc) return finish(rc);
                spare = ModeSolver::pick({in});
                vb = ModeSolver::pick({in, spare});
                kvb = ModeSolver::pick({in, spare, vb});
                // The Jacobi runs to its end (it stops early once the off-diagonal mass is below
                // off_floor) in the interior windows: there a few sweeps leave every Ritz vector a
                // mixture with a large residual even when the block's subspace has converged, and
                // the residuals would never come down to tell.  At the ends of the spectrum, as in
                // tyee_mesh_modes, once the best pair is near the tolerance.
                double best_res = HUGE_VAL;
                for (int64_t c = 0; c < nb; ++c) best_res = std::min(best_res, res[c]);
                const int sweeps = mode == kSquared || best_res <= kNearTol * res_tol ? kJacobiSweeps : kMidSweeps;
                rc = sv.rayleigh_ritz(in, spare, vb, kvb, ritz, sweeps, off_floor);
                if (!rc) rc = sv.residuals(vb, kvb, res);
                if (rc) return finish(rc);
                st.applies += 1;
            }
            // the window's pairs, ascending, to their places in the outputs
            std::vector<double> acc_val(acc.size());
            for (size_t i = 0; i < acc.size(); ++i) acc_val[i] = lam_of(acc[i]);
            // locked: the accepted columns; kept for the next window's start: the trusted pairs
            // beyond the boundary (every other column restarts at random: an unconverged column
            // may lie almost in the span of the deflated modes)
            std::fill(hcols.begin() + nb, hcols.begin() + 2 * nb, 0);
            std::fill(hcols.begin() + 2 * nb, hcols.end(), 1);
            for (int64_t c : acc) hcols[nb + c] = 1;
            for (int64_t c : warm) hcols[2 * nb + c] = 0;
            const bool finished = low + high + int64_t(acc.size()) == nt;
            const int64_t row0 = mode == kTop ? nt - int64_t(acc.size()) : low;
            rc = accept_outputs(acc, acc_val, row0, vb);
            if (rc) return finish(rc);
            if (mode == kTop) {
                high = int64_t(acc.size());
                lam_hi = acc_val.back() + 2.0 * res_tol;   // lambda_max, and the Ritz error above it
                beta_top = finished ? HUGE_VAL : new_bound;
            } else {
                low += int64_t(acc.size());
                if (!finished) {
                    beta = new_bound;
                    for (int64_t c = 0; c < nb; ++c) {        // the block's reach at its end
                        const double z = mode == kSquared ? ritz[c] - sigma : ritz[c];
                        mu[c] = res[c] * res[c] + z * z;
                    }
                    double reach2 = reach_of(mu, a_used);
                    // window 1's block spans [0, R0]; a ball about sigma = beta + R/4 holds as
                    // many modes above beta when 1.25 R = R0.  A later window's ball held some
                    // modes below its beta that the next start block has deflated: the next ball
                    // reaches further.
                    reach2 *= mode == kLinear ? 0.64 : 1.5;
                    sigma = beta + kSigmaAt * std::sqrt(reach2);
                    a_hint = reach2;
                    // lock the accepted columns for deflation, in the ring of kLocked windows
                    TYEE_HIP(hipMemcpyAsync(sv.xb[next_slot].p, sv.B(vb), size_t(nt) * nb * sizeof(double),
                                            hipMemcpyDeviceToDevice, sv.st));
                    hipLaunchKernelGGL(k_keep_columns, dim3(sv.grid_items()), dim3(kBlock), 0, sv.st, sv.n, sv.nb,
                                       sv.cols.as<int32_t>() + nb, sv.xb[next_slot].as<double>());
                    TYEE_HIP(hipGetLastError());
                    if (std::find(locked.begin(), locked.end(), next_slot) == locked.end()) locked.push_back(next_slot);
                    next_slot = (next_slot + 1) % kLocked;
                }
            }
            st.found = low + high;
            st.windows = win + 1;
            st.min_gap = std::isfinite(min_gap) ? min_gap : 0.0;
        }
        return finish(TYEE_OK);
    } catch (const std::bad_alloc &) {
        return fail(TYEE_ENOMEM, "host allocation failed");
    }
}
