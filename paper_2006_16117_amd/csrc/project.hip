// Projection X = V_m Y of the quadrature sums back to C^n (Sec. 2, eq. (reduced);
// the full-space vectors P_R f of the RIM-C indicator, eq. (ISPf)).
//
// Complex GEMM on the FP64 matrix cores through a real embedding: with
// K = 2m real inner index (k, part) and 2c real output columns (j, outpart),
//   X_real(i, (j,o)) = sum_{(k,p)} V_real(i, (k,p)) Ybig((k,p), (j,o)),
//   Ybig = [[Yr, Yi], [-Yi, Yr]]  (per (k, j) 2x2 block).
// Each wavefront computes X^T tiles with v_mfma_f64_16x16x4f64: the 16 columns of
// the instruction's output span 16 consecutive rows i of X, so every lane ends up
// with both parts of X(i, j) for two columns j and stores 16-byte complex values,
// contiguous across lanes.  The wavefront's 16-row panel of V stays in registers
// (one double per lane per 4-deep K step) while Y streams from LDS.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PJ_THREADS = 256;
constexpr int PJ_WAVES = PJ_THREADS / 64;
constexpr int MAXQ = 64;          // K steps of 4 reals (2 complex): m <= 128
constexpr int YCOLS = 64;         // columns of Y staged in LDS at a time

}  // namespace

__global__ __launch_bounds__(PJ_THREADS) void k_vmy(int64_t n, int m, const cplx* __restrict__ V, int64_t ldv,
                                                    const cplx* __restrict__ Y, int64_t ldy, int64_t c,
                                                    cplx* __restrict__ X, double* __restrict__ colpart) {
    extern __shared__ cplx Ys[];   // m x YCOLS
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, kq = lane >> 4;
    const int64_t wg_wave = (int64_t)blockIdx.x * PJ_WAVES + wave;
    const int64_t i0 = wg_wave * 16;
    const int64_t i = i0 + li;
    const int nq = (m + 1) / 2;

    // V panel: lane (li, kq) holds V(i, k = 2q + kq/2), part kq%2, for each q
    double vreg[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        double v = 0.0;
        const int k = 2 * q + (kq >> 1);
        if (q < nq && k < m && i < n) {
            const cplx x = V[i + (int64_t)k * ldv];
            v = (kq & 1) ? x.im : x.re;
        }
        vreg[q] = v;
    }

    for (int64_t s0 = 0; s0 < c; s0 += YCOLS) {
        const int sc = (int)min((int64_t)YCOLS, c - s0);
        __syncthreads();
        for (int e = threadIdx.x; e < m * YCOLS; e += PJ_THREADS) {
            const int k = e % m, jj = e / m;
            Ys[e] = (jj < sc) ? Y[k + (s0 + jj) * ldy] : mk(0.0, 0.0);
        }
        __syncthreads();
        // four independent 8-column tiles per pass, so that four accumulation chains
        // of dependent MFMAs interleave
        for (int jt = 0; jt < sc; jt += 32) {
            // The f64 16x16x4 instruction leaves output row jj of the tile in register jj/4 of the lanes
            // with lane/16 = jj%4.  Row jj of the A operand (= Ybig^T tile, lane row li) is therefore
            // mapped to column j = jt + 8u + 2 (jj%4) + (jj/4)/2 and part (jj/4)%2, so that lane group kq
            // ends up holding (re, im) of columns jt + 8u + 2 kq and jt + 8u + 2 kq + 1 in registers 0..3.
            // A operand: k = 2q + kq/2, part kq%2.
            const int jl0 = jt + 2 * (li & 3) + ((li >> 2) >> 1);
            const int op = (li >> 2) & 1;
            const int pp = kq & 1;
            d4 acc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                if (q < nq) {
                    const int k = 2 * q + (kq >> 1);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int jloc = jl0 + 8 * u;
                        double a = 0.0;
                        if (k < m && jloc < sc) {
                            const cplx y = Ys[k + jloc * m];
                            a = (pp == 0) ? (op == 0 ? y.re : y.im) : (op == 0 ? -y.im : y.re);
                        }
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, vreg[q], acc[u], 0, 0, 0);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                // acc[u]: lane (li, kq), reg r -> tile row jj = kq + 4 r: column j = jt + 8u + 2 kq + r/2,
                // part r%2; tile column li -> row i of X.
                const int jc = jt + 8 * u + 2 * kq;
                const int64_t jA = s0 + jc;
                const int64_t jB = jA + 1;
                const cplx xa = mk(acc[u][0], acc[u][1]);
                const cplx xb = mk(acc[u][2], acc[u][3]);
                if (i < n) {
                    if (jc < sc) X[i + jA * n] = xa;
                    if (jc + 1 < sc) X[i + jB * n] = xb;
                }
                if (colpart != nullptr) {
                    double pa = (i < n) ? norm2(xa) : 0.0;
                    double pb = (i < n) ? norm2(xb) : 0.0;
                    // sum over the 16 rows (lanes li = 0..15 of the same kq group)
#pragma unroll
                    for (int msk = 8; msk >= 1; msk >>= 1) {
                        pa += __shfl_xor(pa, msk, 64);
                        pb += __shfl_xor(pb, msk, 64);
                    }
                    if (li == 0) {
                        if (jc < sc) colpart[wg_wave * c + jA] = pa;
                        if (jc + 1 < sc) colpart[wg_wave * c + jB] = pb;
                    }
                }
            }
        }
    }
}

// Column norms from the per-wave partial sums: first CN_GROUPS groups of waves
// each reduce their share for 64 columns (4 threads per column, LDS combine),
// then one pass adds the groups and takes the square root.
constexpr int CN_GROUPS = 32;

__global__ __launch_bounds__(256) void k_colnorm_partial(const double* __restrict__ colpart, int64_t nwaves, int64_t c,
                                                         double* __restrict__ part) {
    __shared__ double red[4][64];
    const int jl = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + jl;
    const int64_t per = (nwaves + CN_GROUPS - 1) / CN_GROUPS;
    const int64_t w0 = (int64_t)blockIdx.y * per, w1 = min(nwaves, w0 + per);
    double a0 = 0.0, a1 = 0.0;
    if (j < c) {
        int64_t w = w0 + sub;
        for (; w + 4 < w1; w += 8) {
            a0 += colpart[w * c + j];
            a1 += colpart[(w + 4) * c + j];
        }
        if (w < w1) a0 += colpart[w * c + j];
    }
    red[sub][jl] = a0 + a1;
    __syncthreads();
    if (sub == 0 && j < c) part[(int64_t)blockIdx.y * c + j] = red[0][jl] + red[1][jl] + red[2][jl] + red[3][jl];
}

__global__ void k_colnorm_finish(const double* __restrict__ part, int64_t c, double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c) return;
    double acc = 0.0;
    for (int g = 0; g < CN_GROUPS; ++g) acc += part[(int64_t)g * c + j];
    out[j] = sqrt(acc);
}

int64_t project_scratch_elems(int64_t n, int64_t c) {
    const int64_t nwaves = ((n + 15) / 16 + PJ_WAVES - 1) / PJ_WAVES * PJ_WAVES;
    return (nwaves + CN_GROUPS) * c;
}

simm_status project(int64_t n, int m, const cplx* V, int64_t ldv, const cplx* Y, int64_t ldy, int64_t c, cplx* X,
                    double* col_norms, double* scratch, int64_t scratch_elems, hipStream_t st) {
    if (c <= 0) return SIMM_OK;
    if (m < 1 || m > 2 * MAXQ) {
        set_error("Krylov dimension outside 1..128");
        return SIMM_EUNSUPPORTED;
    }
    const int64_t nw = (n + 15) / 16;
    const int64_t nblk = (nw + PJ_WAVES - 1) / PJ_WAVES;
    if (col_norms != nullptr && scratch_elems < (nblk * PJ_WAVES + CN_GROUPS) * c) {
        set_error("projection scratch too small");
        return SIMM_EINVAL;
    }
    const size_t lds = sizeof(cplx) * (size_t)m * YCOLS;
    hipLaunchKernelGGL(k_vmy, dim3((unsigned)nblk), dim3(PJ_THREADS), lds, st, n, m, V, ldv, Y, ldy, c, X,
                       col_norms ? scratch : nullptr);
    if (col_norms != nullptr) {
        double* part = scratch + nblk * PJ_WAVES * c;
        hipLaunchKernelGGL(k_colnorm_partial, dim3((unsigned)((c + 63) / 64), CN_GROUPS), dim3(256), 0, st,
                           (const double*)scratch, nblk * PJ_WAVES, c, part);
        hipLaunchKernelGGL(k_colnorm_finish, dim3((unsigned)((c + 127) / 128)), dim3(128), 0, st,
                           (const double*)part, c, col_norms);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
