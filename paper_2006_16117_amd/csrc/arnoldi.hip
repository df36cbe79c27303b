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
constexpr int GS_MAXCOL = 130;   // Krylov dimension <= 128: at most m + 1 basis columns

__device__ inline cplx shfl_xor_c(cplx v, int mask) {
    return mk(__shfl_xor(v.re, mask, 64), __shfl_xor(v.im, mask, 64));
}

__device__ inline cplx wave_sum(cplx v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = v + shfl_xor_c(v, m);
    return v;
}

// Partial sums over the rows c0 .. c0 + len - 1 staged in ws: column i < ndots gets
// sum conj(V(r, i)) w(r), column ndots (if with_norm) sum |w(r)|^2.  Each wave takes 4
// columns at a time, so that 4 independent load streams are in flight; per column the
// operation order (lanes over rows, then the wave sum) is that of one column at a time.
__device__ inline void chunk_dots(const cplx* __restrict__ V, int64_t ldv, int64_t c0, int len, const cplx* ws,
                                  int ndots, int with_norm, cplx* dst, bool first) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = GS_THREADS / 64;
    const int ntot = ndots + (with_norm ? 1 : 0);
    for (int ib = 4 * wave; ib < ntot; ib += 4 * nw) {
        cplx acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = mk(0.0, 0.0);
        for (int r = lane; r < len; r += 64) {
            const cplx x = ws[r];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = ib + u;
                if (i < ndots) acc[u] = fma_cj(acc[u], V[c0 + r + (int64_t)i * ldv], x);
                else if (i == ndots) acc[u].re += norm2(x);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const cplx t = wave_sum(acc[u]);
            if (lane == 0 && ib + u < ntot) dst[ib + u] = first ? t : dst[ib + u] + t;
        }
    }
}


}  // namespace

// partial[blk * ldp + i] = sum over the block's rows of conj(V(r, i)) * w(r), i < ncol;
// if with_norm, partial[blk * ldp + ncol] = sum |w(r)|^2 (real part).
__device__ __forceinline__ void gs_dots_body(int64_t n, const cplx* __restrict__ V, int64_t ldv, int ncol,
                                             const cplx* __restrict__ w, int with_norm, cplx* partial, int ldp,
                                             cplx* ws) {
    const int64_t nblk = gridDim.x;
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = blockIdx.x * rows;
    const int64_t r1 = min(n, r0 + rows);
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
        chunk_dots(V, ldv, c0, (int)(c1 - c0), ws, ncol, with_norm, partial + blockIdx.x * (int64_t)ldp, c0 == r0);
    }
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_dots(int64_t n, const cplx* __restrict__ V, int64_t ldv, int ncol,
                                                        const cplx* __restrict__ w, int with_norm, cplx* partial,
                                                        int ldp, const int* active) {
    if (active != nullptr && *active == 0) return;
    __shared__ cplx ws[1024];
    gs_dots_body(n, V, ldv, ncol, w, with_norm, partial, ldp, ws);
}

// out[i] = sum_blk partial[blk * ldp + i] for i < ntot: one block per column, a
// fixed-shape tree over the (<= 256) row blocks, so the order never changes.
__device__ __forceinline__ void gs_reduce_body(const cplx* partial, int nblk, int ldp, int ntot, cplx* out,
                                               cplx* red) {
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

__global__ __launch_bounds__(256) void k_gs_reduce(const cplx* partial, int nblk, int ldp, int ntot, cplx* out,
                                                   const int* active) {
    if (active != nullptr && *active == 0) return;
    __shared__ cplx red[256];
    gs_reduce_body(partial, nblk, ldp, ntot, out, red);
}

// One Gram-Schmidt update fused with the partial sums of the next pass, over the same
// row partition as k_gs_dots: w(r) -= sum_{i < ncol} V(r, i) h(i) for the block's rows
// (one thread per row, columns in order), then, on the updated rows, the partial sums
// of conj(V(r, i)) w(r) for i < ndots and, if with_norm, of |w(r)|^2 (as k_gs_dots).
// Saves a launch and a pass over w per update.
__device__ __forceinline__ void gs_update_dots_body(int64_t n, const cplx* __restrict__ V, int64_t ldv, int ncol,
                                                    const cplx* __restrict__ h, cplx* __restrict__ w, int ndots,
                                                    int with_norm, cplx* partial, int ldp, cplx* ws, cplx* hs) {
    const int64_t nblk = gridDim.x;
    const int64_t rows = (n + nblk - 1) / nblk;
    const int64_t r0 = blockIdx.x * rows;
    const int64_t r1 = min(n, r0 + rows);
    const int ntot = ndots + (with_norm ? 1 : 0);
    if (r0 >= r1) {
        for (int i = threadIdx.x; i < ntot; i += GS_THREADS) partial[blockIdx.x * (int64_t)ldp + i] = mk(0.0, 0.0);
        return;
    }
    for (int i = threadIdx.x; i < ncol; i += GS_THREADS) hs[i] = h[i];
    for (int64_t c0 = r0; c0 < r1; c0 += 1024) {
        const int64_t c1 = min(r1, c0 + 1024);
        __syncthreads();
        for (int64_t r = c0 + threadIdx.x; r < c1; r += GS_THREADS) {
            cplx acc = w[r];
            for (int i = 0; i < ncol; ++i) acc = fms(acc, V[r + (int64_t)i * ldv], hs[i]);
            w[r] = acc;
            ws[r - c0] = acc;
        }
        __syncthreads();
        chunk_dots(V, ldv, c0, (int)(c1 - c0), ws, ndots, with_norm, partial + blockIdx.x * (int64_t)ldp, c0 == r0);
    }
}

__global__ __launch_bounds__(GS_THREADS) void k_gs_update_dots(int64_t n, const cplx* __restrict__ V, int64_t ldv,
                                                               int ncol, const cplx* __restrict__ h,
                                                               cplx* __restrict__ w, int ndots, int with_norm,
                                                               cplx* partial, int ldp, const int* active) {
    if (active != nullptr && *active == 0) return;
    __shared__ cplx ws[1024];
    __shared__ cplx hs[GS_MAXCOL];
    gs_update_dots_body(n, V, ldv, ncol, h, w, ndots, with_norm, partial, ldp, ws, hs);
}

// The reduction of ||w||^2 (as k_gs_reduce, one column) and the end of step j:
// H(0..j, j) = h1 + h2, h_{j+1,j} = ||w||, breakdown test against ||M v_j|| (h1[j+1]
// holds its square).
__device__ __forceinline__ void gs_norm_finalize_body(const cplx* partial, int nblk, int j, const cplx* h1,
                                                      const cplx* h2, cplx* hw, cplx* H, int ldh, double* hnorm,
                                                      int* active, int* m_eff, cplx* red) {
    cplx acc = mk(0.0, 0.0);
    for (int b = threadIdx.x; b < nblk; b += 256) acc = acc + partial[b];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    for (int i = threadIdx.x; i <= j; i += blockDim.x) H[i + (int64_t)j * ldh] = h1[i] + h2[i];
    if (threadIdx.x == 0) {
        hw[0] = red[0];
        const double wn = sqrt(red[0].re);
        const double w0 = sqrt(h1[j + 1].re);
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

__global__ __launch_bounds__(256) void k_gs_norm_finalize(const cplx* partial, int nblk, int j, const cplx* h1,
                                                          const cplx* h2, cplx* hw, cplx* H, int ldh, double* hnorm,
                                                          int* active, int* m_eff) {
    if (*active == 0) return;
    __shared__ cplx red[256];
    gs_norm_finalize_body(partial, nblk, j, h1, h2, hw, H, ldh, hnorm, active, m_eff, red);
}

// The same kernels for up to four independent Arnoldi processes at once (same n, j and
// layout; space blockIdx.y), each space's arithmetic exactly that of the kernels above.
__global__ __launch_bounds__(GS_THREADS) void k_gs_dots_b(int64_t n, GsBatch b, int64_t ldv, int ncol, int with_norm,
                                                          int ldp) {
    const int y = blockIdx.y;
    if (*b.active[y] == 0) return;
    __shared__ cplx ws[1024];
    gs_dots_body(n, b.V[y], ldv, ncol, b.V[y] + (int64_t)ncol * ldv, with_norm, b.partial[y], ldp, ws);
}
__global__ __launch_bounds__(256) void k_gs_reduce_b(GsBatch b, int nblk, int ldp, int ntot, int which) {
    const int y = blockIdx.y;
    if (*b.active[y] == 0) return;
    __shared__ cplx red[256];
    gs_reduce_body(b.partial[y], nblk, ldp, ntot, which == 1 ? b.h1[y] : b.h2[y], red);
}
__global__ __launch_bounds__(GS_THREADS) void k_gs_update_dots_b(int64_t n, GsBatch b, int64_t ldv, int ncol, int which,
                                                                 int ndots, int with_norm, int ldp) {
    const int y = blockIdx.y;
    if (*b.active[y] == 0) return;
    __shared__ cplx ws[1024];
    __shared__ cplx hs[GS_MAXCOL];
    gs_update_dots_body(n, b.V[y], ldv, ncol, which == 1 ? b.h1[y] : b.h2[y], b.V[y] + (int64_t)ncol * ldv, ndots,
                        with_norm, b.partial[y], ldp, ws, hs);
}
__global__ __launch_bounds__(256) void k_gs_norm_finalize_b(GsBatch b, int nblk, int j, int ldh) {
    const int y = blockIdx.y;
    if (*b.active[y] == 0) return;
    __shared__ cplx red[256];
    gs_norm_finalize_body(b.partial[y], nblk, j, b.h1[y], b.h2[y], b.h2[y] + (j + 2), b.H[y], ldh, b.hnorm[y],
                          b.active[y], b.m_eff[y], red);
}
__global__ void k_scale_div_b(int64_t n, GsBatch b, int64_t ldv, int col) {
    const int y = blockIdx.y;
    if (*b.active[y] == 0) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    cplx* v = b.V[y] + (int64_t)col * ldv;
    const double s = *b.hnorm[y];
    const cplx x = v[r];
    v[r] = mk(x.re / s, x.im / s);
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
    // w -= V h1, then the partial sums of pass 2 (re-orthogonalisation) on the new w
    hipLaunchKernelGGL(k_gs_update_dots, dim3(w.nblk), dim3(GS_THREADS), 0, st, n, (const cplx*)V, ldv, ncol,
                       (const cplx*)w.h1, wv, ncol, 0, w.partial, ldp, (const int*)active);
    hipLaunchKernelGGL(k_gs_reduce, dim3(ncol), dim3(256), 0, st, (const cplx*)w.partial, w.nblk, ldp, ncol, w.h2,
                       (const int*)active);
    // w -= V h2, then ||w||^2
    hipLaunchKernelGGL(k_gs_update_dots, dim3(w.nblk), dim3(GS_THREADS), 0, st, n, (const cplx*)V, ldv, ncol,
                       (const cplx*)w.h2, wv, 0, 1, w.partial, 1, (const int*)active);
    cplx* hw = w.h2 + (ncol + 1);
    hipLaunchKernelGGL(k_gs_norm_finalize, dim3(1), dim3(256), 0, st, (const cplx*)w.partial, w.nblk, j,
                       (const cplx*)w.h1, (const cplx*)w.h2, hw, H, ldh, w.hnorm, active, m_eff);
    hipLaunchKernelGGL(k_scale_div, dim3(blocks), dim3(256), 0, st, n, wv, (const double*)w.hnorm, (const int*)active);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// Gram-Schmidt part of step j for nr <= 4 spaces at once: w = V_r(:, j+1) holds M v_j of
// space r; per space the operations of arnoldi_step.
simm_status arnoldi_step_batch(int64_t n, const GsBatch& b, int nr, int64_t ldv, int j, int ldh, int nblk,
                               hipStream_t st) {
    const int ncol = j + 1;
    const int ldp = ncol + 1;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    const unsigned y = (unsigned)nr;
    hipLaunchKernelGGL(k_gs_dots_b, dim3(nblk, y), dim3(GS_THREADS), 0, st, n, b, ldv, ncol, 1, ldp);
    hipLaunchKernelGGL(k_gs_reduce_b, dim3(ncol + 1, y), dim3(256), 0, st, b, nblk, ldp, ncol + 1, 1);
    hipLaunchKernelGGL(k_gs_update_dots_b, dim3(nblk, y), dim3(GS_THREADS), 0, st, n, b, ldv, ncol, 1, ncol, 0, ldp);
    hipLaunchKernelGGL(k_gs_reduce_b, dim3(ncol, y), dim3(256), 0, st, b, nblk, ldp, ncol, 2);
    hipLaunchKernelGGL(k_gs_update_dots_b, dim3(nblk, y), dim3(GS_THREADS), 0, st, n, b, ldv, ncol, 2, 0, 1, 1);
    hipLaunchKernelGGL(k_gs_norm_finalize_b, dim3(1, y), dim3(256), 0, st, b, nblk, j, ldh);
    hipLaunchKernelGGL(k_scale_div_b, dim3(blocks, y), dim3(256), 0, st, n, b, ldv, j + 1);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
