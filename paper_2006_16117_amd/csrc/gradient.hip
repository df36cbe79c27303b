// Device pieces of the adjoint gradient of J = sum_R ||x_R||^2, x_R the fine-rule
// projection of f onto the square R (Sec. 2 eq. (XLXf) with the Krylov reduction of
// eq. (reduced)).  With c_j = w_j / (2 pi i), u_j = (A - z_j B)^{-1} f ~ V y_j and
// lambda_j = (A - z_j B)^{-H} x_R ~ V' y'_j (V', y'_j from the conjugate-transposed
// pencil, started from x_R), differentiating the resolvent gives
//   dJ = -2 Re sum_R sum_j c_j lambda_j^H dA u_j,
// so with K_R = sum_j c_j y_j y'_j^H (m x m'), Z = V K_R and Z1 = (A1 V) K_R:
//   dJ/dp                     = -2 Re sum_R sum_i sum_a conj(V'_ia) Z1_ia,
//   dJ/dRe A_ii + i dJ/dIm A_ii = -2 conj( sum_R sum_a conj(V'_ia) Z_ia ).
// The m x m' matrices come from small kernels; Z and Z1 are FP64 MFMA products
// (project.hip); the row-wise dots stream V', Z, Z1 once.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {
constexpr int GR_THREADS = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
}  // namespace

// Band of C^H from the band of C (column-major, leading dimension kl + ku + 1, entry
// (i, c) at row ku + i - c): C^H has kl' = ku, ku' = kl and the same leading dimension.
__global__ void k_conj_transpose_band(int64_t n, int kl, int ku, const cplx* __restrict__ in, cplx* __restrict__ out) {
    const int ld = kl + ku + 1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)ld * n) return;
    const int r = (int)(e % ld);        // row in the band of C^H: ku' + i - c = kl + i - c
    const int64_t c = e / ld;
    const int64_t i = c + r - kl;       // C^H(i, c) = conj(C(c, i))
    cplx v = mk(0.0, 0.0);
    if (i >= 0 && i < n) v = conj(in[(int64_t)(kl + ku - r) + i * ld]);
    out[e] = v;
}

simm_status conj_transpose_band(int64_t n, int kl, int ku, const cplx* in, cplx* out, hipStream_t st) {
    const int64_t total = (int64_t)(kl + ku + 1) * n;
    hipLaunchKernelGGL(k_conj_transpose_band, dim3((unsigned)((total + GR_THREADS - 1) / GR_THREADS)),
                       dim3(GR_THREADS), 0, st, n, kl, ku, in, out);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// K(b, a) = sum_j c_j Yf(j, b) conj(Ya(j, a)), column-major mf x ma, rows of Yf / Ya
// strided by ldy.  The sum runs over j in order.
__global__ void k_grad_kmat(int nf, const cplx* __restrict__ Yf, const cplx* __restrict__ Ya, int ldy,
                            const cplx* __restrict__ cw, int mf, int ma, cplx* __restrict__ K) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mf * ma) return;
    const int b = e % mf, a = e / mf;
    cplx acc = mk(0.0, 0.0);
    for (int j = 0; j < nf; ++j) acc = fma_c(acc, cw[j], Yf[(int64_t)j * ldy + b] * conj(Ya[(int64_t)j * ldy + a]));
    K[e] = acc;
}

simm_status grad_kmat(int nf, const cplx* Yf, const cplx* Ya, int ldy, const cplx* cw, int mf, int ma, cplx* K,
                      hipStream_t st) {
    const int total = mf * ma;
    hipLaunchKernelGGL(k_grad_kmat, dim3((unsigned)((total + GR_THREADS - 1) / GR_THREADS)), dim3(GR_THREADS), 0, st,
                       nf, Yf, Ya, ldy, cw, mf, ma, K);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// Row-wise dots of one square: thread i forms sum_a conj(V'_ia) Z1_ia (summed over the
// workgroup into part[2 blk]) and |x_i|^2 (into part[2 blk + 1]), and adds
// -2 conj(sum_a conj(V'_ia) Z_ia) to grad[i].  Z1 and grad may be null.
__global__ __launch_bounds__(GR_THREADS) void k_grad_rowdot(int64_t n, int ma, const cplx* __restrict__ Vp,
                                                            int64_t ldv, const cplx* __restrict__ Z,
                                                            const cplx* __restrict__ Z1, int64_t ldz,
                                                            const cplx* __restrict__ x, cplx* __restrict__ grad,
                                                            cplx* __restrict__ part) {
    __shared__ double red[3][GR_THREADS / 64];
    const int64_t i = (int64_t)blockIdx.x * GR_THREADS + threadIdx.x;
    cplx s1 = mk(0.0, 0.0);
    double xn = 0.0;
    if (i < n) {
        cplx s = mk(0.0, 0.0);
        for (int a = 0; a < ma; ++a) {
            const cplx v = Vp[i + (int64_t)a * ldv];
            if (grad != nullptr) s = fma_cj(s, v, Z[i + (int64_t)a * ldz]);
            if (Z1 != nullptr) s1 = fma_cj(s1, v, Z1[i + (int64_t)a * ldz]);
        }
        if (grad != nullptr) {
            const cplx gi = grad[i];
            grad[i] = mk(gi.re - 2.0 * s.re, gi.im + 2.0 * s.im);
        }
        xn = norm2(x[i]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double a0 = wave_sum(s1.re), a1 = wave_sum(s1.im), a2 = wave_sum(xn);
    if (lane == 0) {
        red[0][wave] = a0;
        red[1][wave] = a1;
        red[2][wave] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0;
        for (int w = 0; w < GR_THREADS / 64; ++w) {
            r0 += red[0][w];
            r1 += red[1][w];
            r2 += red[2][w];
        }
        part[2 * (int64_t)blockIdx.x] = mk(r0, r1);
        part[2 * (int64_t)blockIdx.x + 1] = mk(r2, 0.0);
    }
}

// acc[0] += sum of the |x|^2 partials, acc[1] += -2 Re(sum of the Z1 partials); one
// wavefront, partials summed in a fixed order.
__global__ void k_grad_finish(int64_t nblk, const cplx* __restrict__ part, double* __restrict__ acc) {
    const int lane = threadIdx.x;
    double s = 0.0, x = 0.0;
    for (int64_t b = lane; b < nblk; b += 64) {
        s += part[2 * b].re;
        x += part[2 * b + 1].re;
    }
    s = wave_sum(s);
    x = wave_sum(x);
    if (lane == 0) {
        acc[0] += x;
        acc[1] += -2.0 * s;
    }
}

simm_status grad_rowdot(int64_t n, int ma, const cplx* Vp, int64_t ldv, const cplx* Z, const cplx* Z1, int64_t ldz,
                        const cplx* x, cplx* grad, cplx* part, double* acc, hipStream_t st) {
    const int64_t nblk = (n + GR_THREADS - 1) / GR_THREADS;
    hipLaunchKernelGGL(k_grad_rowdot, dim3((unsigned)nblk), dim3(GR_THREADS), 0, st, n, ma, Vp, ldv, Z, Z1, ldz, x,
                       grad, part);
    SIMM_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_grad_finish, dim3(1), dim3(64), 0, st, nblk, (const cplx*)part, acc);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// grad = sum over the W per-worker diagonal gradients, in worker order (grad may be
// null); acc[0], acc[1] += the other workers' (J, dJ/dp) pairs acc[2w], acc[2w + 1].
__global__ void k_grad_combine(int64_t n, int W, const cplx* __restrict__ grads, cplx* __restrict__ grad,
                               double* __restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * GR_THREADS + threadIdx.x;
    if (grad != nullptr && i < n) {
        cplx s = grads[i];
        for (int w = 1; w < W; ++w) s = s + grads[(int64_t)w * n + i];
        grad[i] = s;
    }
    if (i == 0) {
        double a = acc[0], b = acc[1];
        for (int w = 1; w < W; ++w) {
            a += acc[2 * w];
            b += acc[2 * w + 1];
        }
        acc[0] = a;
        acc[1] = b;
    }
}

simm_status grad_combine(int64_t n, int W, const cplx* grads, cplx* grad, double* acc, hipStream_t st) {
    const int64_t nblk = grad != nullptr ? (n + GR_THREADS - 1) / GR_THREADS : 1;
    hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)nblk), dim3(GR_THREADS), 0, st, n, W, grads, grad, acc);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

int64_t grad_part_elems(int64_t n) { return 2 * ((n + GR_THREADS - 1) / GR_THREADS); }

}  // namespace simm
