// Lowest eigenmodes of the B-field operator K = -L_E L_B (Section 2: eigenvectors of the
// Maxwell operator in metric (7) and the "complex time" method), on the device in FP64.
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
//   * deflation: the filtered block is made S-orthonormal (Cholesky QR three times, the first
//     with a small diagonal shift: shifted CholeskyQR3 of Fukaya et al., SIAM J. Sci. Comput.
//     2020), so every vector is orthogonal in metric (7) to the others;
//   * Rayleigh-Ritz: H = V^T S K V is diagonalised (cyclic Jacobi) and V rotated into Ritz
//     vectors; the largest Ritz value of the block becomes the next a.
// b is a Gershgorin bound on lambda_max of the symmetric form S^(1/2) K S^(-1/2).
//
// Layout: the block is row-major, [n_t][nb] doubles (row = triangle in device numbering), so
// the three neighbour rows that a triangle gathers are contiguous runs of nb values.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "sim.hpp"

namespace tyee {
namespace {

constexpr int kMaxBlock = 256;
constexpr int kRotRows = 16;        // rows of the block per work-group in k_rotate
constexpr int kGramTile = 32;       // output tile of k_gram (32 x 32)
constexpr int kGramRows = 64;       // rows staged in LDS per pass of k_gram

// y_out = alpha * (K y) + beta * y + gam * y_prev   (y_prev may be null)
__global__ void k_modes_apply(int32_t n, int32_t nb, const double *__restrict__ y,
                              const double *__restrict__ yp, double *__restrict__ yo,
                              const int32_t *__restrict__ nbr, const double *__restrict__ wt,
                              const double *__restrict__ inv_s, double alpha, double beta, double gam) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= uint32_t(n) * uint32_t(nb)) return;
    const uint32_t j = g / uint32_t(nb), c = g - j * uint32_t(nb);
    const double yj = y[g];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int32_t o = nbr[3 * j + q];
        if (o >= 0) acc += wt[3 * j + q] * (yj - y[uint32_t(o) * uint32_t(nb) + c]);
    }
    double out = alpha * (acc * inv_s[j]) + beta * yj;
    if (yp) out += gam * yp[g];
    yo[g] = out;
}

// partial[chunk][p][q] = sum over the chunk's rows j of S_j x[j][p] z[j][q]
// grid (chunks, tiles_p, tiles_q), 256 threads: a 16 x 16 grid of threads, 2 x 2 outputs each
__global__ void __launch_bounds__(256) k_gram(int32_t n, int32_t nb, int32_t rows_per_chunk,
                                              const double *__restrict__ x, const double *__restrict__ z,
                                              const double *__restrict__ s, double *__restrict__ partial) {
    __shared__ double xs[kGramRows][kGramTile];
    __shared__ double zs[kGramRows][kGramTile];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int p0 = blockIdx.y * kGramTile, q0 = blockIdx.z * kGramTile;
    const int64_t r_begin = int64_t(blockIdx.x) * rows_per_chunk;
    const int64_t r_end = std::min<int64_t>(n, r_begin + rows_per_chunk);
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int64_t r0 = r_begin; r0 < r_end; r0 += kGramRows) {
        for (int e = tid; e < kGramRows * kGramTile; e += 256) {
            const int rr = e / kGramTile, cc = e % kGramTile;
            const int64_t row = r0 + rr;
            const bool in = row < r_end;
            const double sw = in ? s[row] : 0.0;
            xs[rr][cc] = (in && p0 + cc < nb) ? sw * x[row * nb + p0 + cc] : 0.0;
            zs[rr][cc] = (in && q0 + cc < nb) ? z[row * nb + q0 + cc] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < kGramRows; ++rr) {
            const double a0 = xs[rr][ty], a1 = xs[rr][ty + 16];
            const double b0 = zs[rr][tx], b1 = zs[rr][tx + 16];
            acc[0][0] += a0 * b0;
            acc[0][1] += a0 * b1;
            acc[1][0] += a1 * b0;
            acc[1][1] += a1 * b1;
        }
        __syncthreads();
    }
    double *out = partial + size_t(blockIdx.x) * nb * nb;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int p = p0 + ty + 16 * a, q = q0 + tx + 16 * b;
            if (p < nb && q < nb) out[p * nb + q] = acc[a][b];
        }
}

// out[k] = sum over chunks c (in order) of partial[c][k]
__global__ void k_sum_chunks(int32_t chunks, int32_t len, const double *__restrict__ partial,
                             double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += partial[size_t(c) * len + k];
    out[k] = acc;
}

// y[j][c] = sum_k x[j][k] m[k][c]  (m upper triangular when upper != 0); blockDim >= nb
__global__ void k_rotate(int32_t n, int32_t nb, const double *__restrict__ x, const double *__restrict__ m,
                         double *__restrict__ y, int32_t upper) {
    __shared__ double xs[kRotRows][kMaxBlock];
    const int64_t r0 = int64_t(blockIdx.x) * kRotRows;
    const int rows = int(std::min<int64_t>(kRotRows, n - r0));
    for (int e = threadIdx.x; e < kRotRows * nb; e += blockDim.x) {
        const int rr = e / nb, cc = e % nb;
        xs[rr][cc] = rr < rows ? x[(r0 + rr) * nb + cc] : 0.0;
    }
    __syncthreads();
    const int c = threadIdx.x;
    if (c >= nb) return;
    double acc[kRotRows];
#pragma unroll
    for (int r = 0; r < kRotRows; ++r) acc[r] = 0.0;
    const int kend = upper ? c + 1 : nb;
    for (int k = 0; k < kend; ++k) {
        const double mk = m[k * nb + c];
#pragma unroll
        for (int r = 0; r < kRotRows; ++r) acc[r] += xs[r][k] * mk;
    }
    for (int r = 0; r < rows; ++r) y[(r0 + r) * nb + c] = acc[r];
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
                                                int32_t max_sweeps, int32_t *__restrict__ sweeps_out) {
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
        if (off_sum <= 1e-30 * all_sum || all_sum == 0.0) break;
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
    for (int64_t j = r_begin; j < r_end; ++j) {
        const double r = kv[j * nb + c] - th * v[j * nb + c];
        acc += s[j] * r * r;
    }
    partial[size_t(blockIdx.x) * nb + c] = acc;
}

// x[j][c] = 2 u - 1 with u = (splitmix64(seed + j nb + c) >> 11) 2^-53 (canonical j)
__global__ void k_random_block(int32_t n, int32_t nb, const int32_t *__restrict__ canon, uint64_t seed,
                               double *__restrict__ x) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= uint32_t(n) * uint32_t(nb)) return;
    const uint32_t j = g / uint32_t(nb), c = g - j * uint32_t(nb);
    uint64_t z = seed + uint64_t(canon[j]) * uint64_t(nb) + c + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[g] = 2.0 * (double(z >> 11) * 0x1.0p-53) - 1.0;
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
    hipStream_t st = nullptr;
    DeviceBuffer nbr, wt, inv_s, s, canon;
    DeviceBuffer buf[5];               // block-sized buffers
    DeviceBuffer g, m, h, q, work, theta, partial, small_i;

    double *B(int i) const { return buf[i].as<double>(); }

    int alloc(const Mesh &mesh, const double *gamma, int32_t nblock, double *upper) {
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
        rows_per_chunk = int32_t(std::max<int64_t>(256, (nt + 255) / 256));
        chunks = int32_t((nt + rows_per_chunk - 1) / rows_per_chunk);
        int rc = TYEE_OK;
        for (int i = 0; i < 5 && !rc; ++i) rc = buf[i].alloc(blk);
        if (!rc) rc = nbr.alloc(hn.size() * 4);
        if (!rc) rc = wt.alloc(hw.size() * 8);
        if (!rc) rc = inv_s.alloc(nt * 8);
        if (!rc) rc = s.alloc(nt * 8);
        if (!rc) rc = canon.alloc(nt * 4);
        const size_t sq = size_t(nb) * nb * sizeof(double);
        if (!rc) rc = g.alloc(sq);
        if (!rc) rc = m.alloc(sq);
        if (!rc) rc = h.alloc(sq);
        if (!rc) rc = q.alloc(sq);
        if (!rc) rc = work.alloc(sq);
        if (!rc) rc = theta.alloc(size_t(nb) * 8);
        if (!rc) rc = partial.alloc(size_t(chunks) * nb * nb * sizeof(double));
        if (!rc) rc = small_i.alloc(2 * sizeof(int32_t));
        if (rc) return rc;
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
        hipLaunchKernelGGL(k_modes_apply, dim3(grid_items()), dim3(kBlock), 0, st, n, nb, y, yp, yo,
                           nbr.as<int32_t>(), wt.as<double>(), inv_s.as<double>(), alpha, beta, gam);
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    // out (nb x nb) = x^T S z
    int gram(const double *x, const double *z, double *out) {
        const int tiles = (nb + kGramTile - 1) / kGramTile;
        hipLaunchKernelGGL(k_gram, dim3(chunks, tiles, tiles), dim3(256), 0, st, n, nb, rows_per_chunk, x, z,
                           s.as<double>(), partial.as<double>());
        TYEE_HIP(hipGetLastError());
        const int len = nb * nb;
        hipLaunchKernelGGL(k_sum_chunks, dim3((len + 255) / 256), dim3(256), 0, st, chunks, len,
                           partial.as<double>(), out);
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    int rotate(const double *x, const double *mat, double *y, bool upper) {
        const int threads = ((nb + 63) / 64) * 64;
        hipLaunchKernelGGL(k_rotate, dim3((n + kRotRows - 1) / kRotRows), dim3(threads), 0, st, n, nb, x, mat, y,
                           int32_t(upper));
        TYEE_HIP(hipGetLastError());
        return TYEE_OK;
    }

    // x (in buffer ix) -> S-orthonormal block in buffer iy, by Cholesky QR three times (the
    // first with a small diagonal shift, which keeps the factorisation defined for a block
    // that the filter has made nearly dependent).  Returns TYEE_EUNSTABLE when a
    // factorisation fails.
    int orthonormalise(int ix, int iy) {
        int src = ix, dst = iy;
        for (int pass = 0; pass < 3; ++pass) {
            int rc = gram(B(src), B(src), g.as<double>());
            if (rc) return rc;
            double shift = 0.0;
            if (pass == 0) {
                // shift = 11 (n nb + nb (nb + 1)) u ||G||_2, ||G||_2 bounded by the trace
                std::vector<double> hg(size_t(nb) * nb);
                TYEE_HIP(hipMemcpyAsync(hg.data(), g.p, hg.size() * 8, hipMemcpyDeviceToHost, st));
                TYEE_HIP(hipStreamSynchronize(st));
                double tr = 0.0;
                for (int i = 0; i < nb; ++i) tr += hg[size_t(i) * nb + i];
                shift = 11.0 * (double(n) * nb + double(nb) * (nb + 1)) * 0x1.0p-53 * tr;
            }
            hipLaunchKernelGGL(k_chol_inverse, dim3(1), dim3(256), 0, st, nb, g.as<double>(), shift, m.as<double>(),
                               small_i.as<int32_t>());
            TYEE_HIP(hipGetLastError());
            int32_t info = 0;
            TYEE_HIP(hipMemcpyAsync(&info, small_i.p, 4, hipMemcpyDeviceToHost, st));
            TYEE_HIP(hipStreamSynchronize(st));
            if (info) return fail(TYEE_EUNSTABLE, "mode block lost rank (Cholesky pivot " + std::to_string(info) + ")");
            rc = rotate(B(src), m.as<double>(), B(dst), true);
            if (rc) return rc;
            std::swap(src, dst);
        }
        // three passes: the result sits in iy
        return TYEE_OK;
    }

    // Rayleigh-Ritz of the S-orthonormal block in buffer iv (scratch iz): Ritz vectors to
    // buffer 3, K times them to buffer 4, Ritz values to host.
    int rayleigh_ritz(int iv, int iz, std::vector<double> &ritz) {
        int rc = apply(B(iv), nullptr, B(iz), 1.0, 0.0, 0.0);
        if (!rc) rc = gram(B(iv), B(iz), h.as<double>());
        if (rc) return rc;
        hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(256), 0, st, nb, h.as<double>(), work.as<double>(), q.as<double>(),
                           theta.as<double>(), int32_t(40), small_i.as<int32_t>() + 1);
        TYEE_HIP(hipGetLastError());
        rc = rotate(B(iv), q.as<double>(), B(3), false);
        if (!rc) rc = rotate(B(iz), q.as<double>(), B(4), false);
        if (rc) return rc;
        ritz.resize(nb);
        TYEE_HIP(hipMemcpyAsync(ritz.data(), theta.p, size_t(nb) * 8, hipMemcpyDeviceToHost, st));
        TYEE_HIP(hipStreamSynchronize(st));
        return TYEE_OK;
    }

    int residuals(std::vector<double> &res) {
        hipLaunchKernelGGL(k_residual, dim3(chunks), dim3(((nb + 63) / 64) * 64), 0, st, n, nb, rows_per_chunk,
                           B(3), B(4), theta.as<double>(), s.as<double>(), partial.as<double>());
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

    // Degree-k filter of the block in buffer 3 damping [a, b_up] with a0 the estimate of the
    // lowest eigenvalue; the result lands in buffer *out (one of 0, 1, 2).
    int filter(int degree, double a, double b_up, double a0, int *out) {
        const double e = 0.5 * (b_up - a), c = 0.5 * (b_up + a);
        const double sigma1 = e / (a0 - c);
        double sigma = sigma1;
        // y1 = (sigma1 / e) (K - c) y0
        int rc = apply(B(3), nullptr, B(0), sigma1 / e, -sigma1 * c / e, 0.0);
        if (rc) return rc;
        int prev = 3, cur = 0;
        for (int k = 2; k <= degree; ++k) {
            const double sigma_new = 1.0 / (2.0 / sigma1 - sigma);
            const int nxt = (cur + 1) % 3 == prev ? (cur + 2) % 3 : (cur + 1) % 3;
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

extern "C" int tyee_mesh_modes(const tyee_mesh *mesh, const double *gamma, int64_t n_modes, int32_t block,
                               int32_t degree, double tol, int32_t max_iter, uint64_t seed, void *stream,
                               double *omega2, double *modes, double *residual, tyee_modes_stats *stats) {
    using namespace tyee;
    if (!mesh || !omega2) return fail(TYEE_EINVAL, "null argument");
    const Mesh &msh = mesh->m;
    const int64_t nt = msh.nt;
    if (n_modes < 1 || n_modes > std::min<int64_t>(nt, kMaxBlock))
        return fail(TYEE_EINVAL, "n_modes must be in 1 .. min(n_triangles, 256)");
    int64_t nb = block;
    if (nb == 0) nb = std::min<int64_t>({nt, int64_t(kMaxBlock), n_modes + std::max<int64_t>(16, n_modes / 4)});
    if (nb < std::max<int64_t>(n_modes, 2) || nb > std::min<int64_t>(nt, kMaxBlock))
        return fail(TYEE_EINVAL, "block must be in max(n_modes, 2) .. min(n_triangles, 256)");
    if (nt * nb >= (int64_t(1) << 31)) return fail(TYEE_EINVAL, "n_triangles x block must be below 2^31");
    if (degree == 0) degree = 64;
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
        // random start, S-orthonormalised, then a first Rayleigh-Ritz for the bounds
        hipLaunchKernelGGL(k_random_block, dim3(sv.grid_items()), dim3(kBlock), 0, sv.st, sv.n, sv.nb,
                           sv.canon.as<int32_t>(), seed, sv.B(0));
        TYEE_HIP(hipGetLastError());
        rc = sv.orthonormalise(0, 1);
        std::vector<double> ritz, res;
        if (!rc) rc = sv.rayleigh_ritz(1, 2, ritz);
        if (!rc) rc = sv.residuals(res);
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
            int fo = 0;
            if (filtered) {
                // cap the degree so that the lowest mode grows at most 1e10 times more than
                // the modes at the cut: the filtered block then keeps a condition number that
                // the shifted Cholesky QR recovers from
                const double x0 = (0.5 * (b_up + a) - a0) / (0.5 * (b_up - a));
                int deg = degree;
                if (x0 > 1.0) deg = int(std::max(1.0, std::min(double(degree), std::floor(std::log(2e10) / std::acosh(x0)))));
                TYEE_HIP(hipEventRecord(ev.a, sv.st));
                rc = sv.filter(deg, a, b_up, a0, &fo);
                TYEE_HIP(hipEventRecord(ev.b, sv.st));
                applies += deg;
            } else {
                TYEE_HIP(hipMemcpyAsync(sv.B(0), sv.B(3), size_t(nt) * nb * 8, hipMemcpyDeviceToDevice, sv.st));
            }
            if (rc) break;
            const int other = fo == 0 ? 1 : 0;
            const int spare = 3 - fo - other;      // the third of buffers 0, 1, 2
            rc = sv.orthonormalise(fo, other);
            if (!rc) rc = sv.rayleigh_ritz(other, spare, ritz);
            if (!rc) rc = sv.residuals(res);
            if (rc) break;
            if (filtered) {
                float ms = 0.0f;
                TYEE_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
                filter_ms += ms;
            }
            applies += 1;                          // the Rayleigh-Ritz product K V
            ++it;
            done = converged();
        }
        if (rc) return rc;
        for (int64_t c = 0; c < n_modes; ++c) omega2[c] = ritz[c];
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
            TYEE_HIP(hipMemcpyAsync(hv.data(), sv.B(3), hv.size() * 8, hipMemcpyDeviceToHost, sv.st));
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
