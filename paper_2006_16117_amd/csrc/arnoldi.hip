// Arnoldi process of Sec. 2 on M = (A - sigma B)^{-1} B, one column j at a time:
//   w = M v_j;  h_{1:j,j} = V_j^H w;  w -= V_j h;  (repeated once: classical
//   Gram-Schmidt applied twice);  h_{j+1,j} = ||w||;  v_{j+1} = w / h_{j+1,j};
// with the happy-breakdown stop h_{j+1,j} <= 1e-14 ||M v_j||.
//
// Reductions over the n rows are two-stage and in a fixed order (per-block partial
// sums, then one block summing the partials sequentially), so every run gives
// bitwise the same H.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

constexpr int GS_THREADS = 256;

__device__ inline cplx shfl_xor_c(cplx v, int mask) {
    return mk(__shfl_xor(v.re, mask, 64), __shfl_xor(v.im, mask, 64));
}

__device__ inline cplx wave_sum(cplx v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = v + shfl_xor_c(v, m);
    return v;
}

}  // namespace

// partial[blk * ldp + i] = sum over the block's rows of conj(V(r, i)) * w(r), i < ncol;
// if with_norm, partial[blk * ldp + ncol] = sum |w(r)|^2 (real part).
__global__ __launch_bounds__(GS_THREADS) void k_gs_dots(int64_t n, const cplx* __restrict__ V, int64_t ldv, int ncol,
                                                        const cplx* __restrict__ w, int with_norm, cplx* partial,
                                                        int ldp, const int* active) {
    if (active != nullptr && *active == 0) return;
    __shared__ cplx ws[1024];
    const int64_t nblk = gridDim.x;
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = blockIdx.x * rows;
    const int64_t r1 = min(n, r0 + rows);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = GS_THREADS / 64;
    const int ntot = ncol + (with_norm ? 1 : 0);
    if (r0 >= r1) {
        for (int i = threadIdx.x; i < ntot; i += GS_THREADS) partial[blockIdx.x * (int64_t)ldp + i] = mk(0.0, 0.0);
        return;
    }
    for (int64_t c0 = r0; c0 < r1; c0 += 1024) {
        const int64_t c1 = min(r1, c0 + 1024);
        // (a block handles at most a few thousand rows; chunks of 1024 staged in LDS)
        __syncthreads();
        for (int64_t r = c0 + threadIdx.x; r < c1; r += GS_THREADS) ws[r - c0] = w[r];
        __syncthreads();
        for (int i = wave; i < ntot; i += nw) {
            cplx acc = mk(0.0, 0.0);
            if (i < ncol) {
                const cplx* col = V + (int64_t)i * ldv;
                for (int64_t r = c0 + lane; r < c1; r += 64) acc = fma_cj(acc, col[r], ws[r - c0]);
            } else {
                for (int64_t r = c0 + lane; r < c1; r += 64) acc.re += norm2(ws[r - c0]);
            }
            acc = wave_sum(acc);
            if (lane == 0) {
                cplx* dst = partial + blockIdx.x * (int64_t)ldp + i;
                if (c0 == r0) *dst = acc;
                else *dst = *dst + acc;
            }
        }
    }
}

// out[i] = sum_blk partial[blk * ldp + i] for i < ntot: one block per column, a
// fixed-shape tree over the (<= 256) row blocks, so the order never changes.
__global__ __launch_bounds__(256) void k_gs_reduce(const cplx* partial, int nblk, int ldp, int ntot, cplx* out,
                                                   const int* active) {
    if (active != nullptr && *active == 0) return;
    __shared__ cplx red[256];
    const int i = blockIdx.x;
    if (i >= ntot) return;
    cplx acc = mk(0.0, 0.0);
    for (int b = threadIdx.x; b < nblk; b += 256) acc = acc + partial[(int64_t)b * ldp + i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
}

// w(r) -= sum_{i < ncol} V(r, i) h(i)
__global__ void k_gs_update(int64_t n, const cplx* __restrict__ V, int64_t ldv, int ncol, const cplx* __restrict__ h,
                            cplx* __restrict__ w, const int* active) {
    if (active != nullptr && *active == 0) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    cplx acc = w[r];
    for (int i = 0; i < ncol; ++i) acc = fms(acc, V[r + (int64_t)i * ldv], h[i]);
    w[r] = acc;
}

// H(0..j, j) = h1 + h2, h_{j+1,j} = ||w||, breakdown test; hn0 / hn1 hold sums of squares.
__global__ void k_arnoldi_finalize(int j, const cplx* h1, const cplx* h2, const cplx* hn_w, double hn1_sq,
                                   const cplx* hn1, cplx* H, int ldh, double* hnorm, int* active, int* m_eff) {
    if (*active == 0) return;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) H[i + (int64_t)j * ldh] = h1[i] + h2[i];
    if (threadIdx.x == 0) {
        const double wn = sqrt(hn_w[0].re);
        const double w0 = sqrt(hn1[j + 1].re);
        (void)hn1_sq;
        hnorm[0] = wn;
        hnorm[1] = w0;
        if (wn <= 1e-14 * w0) {
            H[(j + 1) + (int64_t)j * ldh] = mk(0.0, 0.0);
            *active = 0;
            *m_eff = j + 1;
        } else {
            H[(j + 1) + (int64_t)j * ldh] = mk(wn, 0.0);
        }
    }
}

// v = w / s (in place) where s = *hnorm
__global__ void k_scale_div(int64_t n, cplx* v, const double* hnorm, const int* active) {
    if (active != nullptr && *active == 0) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double s = *hnorm;
    const cplx x = v[r];
    v[r] = mk(x.re / s, x.im / s);
}

// beta = ||b||; v1 = b / beta
__global__ void k_norm_finish(const cplx* hsum, double* beta_out) {
    if (threadIdx.x == 0) *beta_out = sqrt(hsum[0].re);
}

simm_status vec_norm_scale(int64_t n, const cplx* b, cplx* v1, double* beta, ArnoldiWork& w, hipStream_t st) {
    const int ldp = 1;
    hipLaunchKernelGGL(k_gs_dots, dim3(w.nblk), dim3(GS_THREADS), 0, st, n, (const cplx*)nullptr, (int64_t)0, 0, b, 1,
                       w.partial, ldp, (const int*)nullptr);
    hipLaunchKernelGGL(k_gs_reduce, dim3(1), dim3(256), 0, st, w.partial, w.nblk, ldp, 1, w.h1, (const int*)nullptr);
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(64), 0, st, w.h1, beta);
    if (v1 != b) SIMM_HIP_TRY(hipMemcpyAsync(v1, b, n * sizeof(cplx), hipMemcpyDeviceToDevice, st));
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_scale_div, dim3(blocks), dim3(256), 0, st, n, v1, (const double*)beta, (const int*)nullptr);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// Gram-Schmidt part of step j: w = V(:, j+1) already holds M v_j.
simm_status arnoldi_step(int64_t n, cplx* V, int64_t ldv, int j, cplx* H, int ldh, ArnoldiWork& w, int* active,
                         int* m_eff, hipStream_t st) {
    cplx* wv = V + (int64_t)(j + 1) * ldv;
    const int ncol = j + 1;
    const int ldp = ncol + 1;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    // pass 1: h1 = V^H w and ||w||^2
    hipLaunchKernelGGL(k_gs_dots, dim3(w.nblk), dim3(GS_THREADS), 0, st, n, (const cplx*)V, ldv, ncol, (const cplx*)wv,
                       1, w.partial, ldp, (const int*)active);
    hipLaunchKernelGGL(k_gs_reduce, dim3(ncol + 1), dim3(256), 0, st, (const cplx*)w.partial, w.nblk, ldp, ncol + 1,
                       w.h1, (const int*)active);
    hipLaunchKernelGGL(k_gs_update, dim3(blocks), dim3(256), 0, st, n, (const cplx*)V, ldv, ncol, (const cplx*)w.h1, wv,
                       (const int*)active);
    // pass 2 (re-orthogonalisation)
    hipLaunchKernelGGL(k_gs_dots, dim3(w.nblk), dim3(GS_THREADS), 0, st, n, (const cplx*)V, ldv, ncol, (const cplx*)wv,
                       0, w.partial, ldp, (const int*)active);
    hipLaunchKernelGGL(k_gs_reduce, dim3(ncol), dim3(256), 0, st, (const cplx*)w.partial, w.nblk, ldp, ncol, w.h2,
                       (const int*)active);
    hipLaunchKernelGGL(k_gs_update, dim3(blocks), dim3(256), 0, st, n, (const cplx*)V, ldv, ncol, (const cplx*)w.h2, wv,
                       (const int*)active);
    // ||w||
    hipLaunchKernelGGL(k_gs_dots, dim3(w.nblk), dim3(GS_THREADS), 0, st, n, (const cplx*)nullptr, (int64_t)0, 0,
                       (const cplx*)wv, 1, w.partial, 1, (const int*)active);
    cplx* hw = w.h2 + (ncol + 1);
    hipLaunchKernelGGL(k_gs_reduce, dim3(1), dim3(256), 0, st, (const cplx*)w.partial, w.nblk, 1, 1, hw,
                       (const int*)active);
    hipLaunchKernelGGL(k_arnoldi_finalize, dim3(1), dim3(128), 0, st, j, (const cplx*)w.h1, (const cplx*)w.h2,
                       (const cplx*)hw, 0.0, (const cplx*)w.h1, H, ldh, w.hnorm, active, m_eff);
    hipLaunchKernelGGL(k_scale_div, dim3(blocks), dim3(256), 0, st, n, wv, (const double*)w.hnorm, (const int*)active);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
