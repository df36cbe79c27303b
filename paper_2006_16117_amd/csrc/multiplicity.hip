// Multiplicities of the computed eigenvalues (Sec. 3.4): per cluster, the
// spectral projections P f_1 .. P f_k of k start vectors are assembled from the
// contour sums of the cluster's level-K squares (Sec. 2, eq. (XLXf) reduced to the
// Krylov space, eq. (reduced)); the number of significant singular values of
// [P f_1 .. P f_k] is the multiplicity.  The device kernels here gather the sums,
// accumulate the projected columns and form the k x k Gram matrices; the
// singular values of a cluster come from the eigenvalues of its Gram matrix
// (a k x k problem, solved on the host by cyclic Jacobi).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {
constexpr int GRAM_THREADS = 256;
}

// Y(:, c) = sum of the fine-rule sums s_f of cluster c's squares:
// rows idx[off[c]] .. idx[off[c+1]-1] of `sums` (each row: s_c then s_f, m_sums each).
__global__ void k_cluster_sums(const cplx* __restrict__ sums, int m_sums, const int64_t* __restrict__ off,
                               const int64_t* __restrict__ idx, int mrows, cplx* __restrict__ Y, int64_t ldy) {
    const int64_t c = blockIdx.x;
    for (int k = threadIdx.x; k < mrows; k += blockDim.x) {
        cplx acc = mk(0.0, 0.0);
        for (int64_t q = off[c]; q < off[c + 1]; ++q) acc = acc + sums[(2 * idx[q] + 1) * (int64_t)m_sums + k];
        Y[k + c * ldy] = acc;
    }
}

// X(:, c) += T(:, c) for c < ncl, X with leading dimension ldx, T with n.
__global__ void k_accum_cols(int64_t n, int64_t ncl, const cplx* __restrict__ T, cplx* __restrict__ X, int64_t ldx) {
    const int64_t total = n * ncl;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, r = e - c * n;
        X[r + c * ldx] = X[r + c * ldx] + T[e];
    }
}

// G(a, b) of cluster c = X_a^H X_b with X_a = column c k + a of X (n rows):
// one workgroup per (c, a, b); strided partial sums, wavefront then LDS reduction.
__global__ __launch_bounds__(GRAM_THREADS) void k_gram(int64_t n, int k, const cplx* __restrict__ X,
                                                        cplx* __restrict__ G) {
    __shared__ double red[2 * (GRAM_THREADS / 64)];
    const int64_t blk = blockIdx.x;
    const int64_t c = blk / ((int64_t)k * k);
    const int a = (int)((blk / k) % k), b = (int)(blk % k);
    const cplx* xa = X + (c * k + a) * n;
    const cplx* xb = X + (c * k + b) * n;
    double re = 0.0, im = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += GRAM_THREADS) {
        const cplx u = xa[r], v = xb[r];
        re += u.re * v.re + u.im * v.im;   // conj(u) v
        im += u.re * v.im - u.im * v.re;
    }
#pragma unroll
    for (int msk = 32; msk >= 1; msk >>= 1) {
        re += __shfl_xor(re, msk, 64);
        im += __shfl_xor(im, msk, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[2 * wave] = re;
        red[2 * wave + 1] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sr = 0.0, si = 0.0;
        for (int w = 0; w < GRAM_THREADS / 64; ++w) {
            sr += red[2 * w];
            si += red[2 * w + 1];
        }
        G[blk] = mk(sr, si);
    }
}

simm_status cluster_sums(const cplx* sums, int m_sums, const int64_t* off, const int64_t* idx, int64_t ncl,
                         int mrows, cplx* Y, int64_t ldy, hipStream_t st) {
    if (ncl <= 0) return SIMM_OK;
    hipLaunchKernelGGL(k_cluster_sums, dim3((unsigned)ncl), dim3(128), 0, st, sums, m_sums, off, idx, mrows, Y, ldy);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status accum_cols(int64_t n, int64_t ncl, const cplx* T, cplx* X, int64_t ldx, hipStream_t st) {
    if (n <= 0 || ncl <= 0) return SIMM_OK;
    const int64_t total = n * ncl;
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_accum_cols, dim3(grid), dim3(256), 0, st, n, ncl, T, X, ldx);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status gram(int64_t n, int k, int64_t ncl, const cplx* X, cplx* G, hipStream_t st) {
    if (ncl <= 0) return SIMM_OK;
    const int64_t blocks = ncl * k * k;
    hipLaunchKernelGGL(k_gram, dim3((unsigned)blocks), dim3(GRAM_THREADS), 0, st, n, k, X, G);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// Eigenvalues of a k x k Hermitian matrix (column-major), descending: cyclic Jacobi
// on its real symmetric embedding [[Re G, -Im G], [Im G, Re G]], whose spectrum is
// that of G with every eigenvalue twice.
std::vector<double> hermitian_eigenvalues(int k, const cplx* G) {
    const int N = 2 * k;
    std::vector<double> S((size_t)N * N);
    auto at = [&](int i, int j) -> double& { return S[(size_t)i + (size_t)j * N]; };
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) {
            const cplx g = G[i + (size_t)j * k];
            at(i, j) = g.re;
            at(i + k, j + k) = g.re;
            at(i + k, j) = g.im;
            at(i, j + k) = -g.im;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) (i == j ? diag : off) += at(i, j) * at(i, j);
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < N - 1; ++p)
            for (int q = p + 1; q < N; ++q) {
                const double apq = at(p, q);
                if (apq == 0.0) continue;
                // rotation zeroing (p, q): tan(2 theta) = 2 a_pq / (a_qq - a_pp)
                const double tau = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < N; ++r) {   // columns p, q
                    const double rp = at(r, p), rq = at(r, q);
                    at(r, p) = c * rp - s * rq;
                    at(r, q) = s * rp + c * rq;
                }
                for (int r = 0; r < N; ++r) {   // rows p, q
                    const double pr = at(p, r), qr = at(q, r);
                    at(p, r) = c * pr - s * qr;
                    at(q, r) = s * pr + c * qr;
                }
            }
    }
    std::vector<double> ev(N);
    for (int i = 0; i < N; ++i) ev[i] = at(i, i);
    std::sort(ev.begin(), ev.end(), [](double a, double b) { return a > b; });
    std::vector<double> out(k);
    for (int i = 0; i < k; ++i) out[i] = 0.5 * (ev[2 * i] + ev[2 * i + 1]);   // the two copies
    return out;
}

}  // namespace simm
