// Application of the Cayley operator M = (A - sigma B)^{-1} B (Sec. 2, eq. (IMxb))
// through the band LU factor: y = U^{-1} L^{-1} P u with u = s B x (or u = f for the
// right-hand side b = (A - sigma B)^{-1} f).
//
// Forward sweep (interleaved L): for j = 0 .. n-1: swap rows j and ipiv[j], then
// rows j+1 .. j+kl -= l(:,j) * row j.  Backward sweep: for j = n-1 .. 0:
// y_j = row_j / u_jj, rows j-kv .. j-1 -= u(:,j) * y_j.
//
// One workgroup per sweep.  The active window of rows lives in registers: thread t
// owns every row i = t (mod W), W = blockDim >= kv + 2, and keeps its row's value
// across column steps.  Only two values cross threads per step -- the pivot row and
// row j -- and they travel through a parity-indexed LDS slot written before the
// step's single barrier.  Each step reads one factor column contiguously; every
// thread issues the same loads each step (factor entry, pivot index, diagonal, next
// input row), PF steps ahead, into register rings.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

constexpr int PF = 8;   // prefetch distance (columns)

struct SweepArgs {
    int64_t n;
    int kl, kv, ldab;
    const cplx* AB;
    const int* ipiv;
    const cplx* u;        // input vector
    const int* active;    // device flag: if *active == 0 the sweep is skipped (NULL: always run)
    cplx* y;              // output (also holds the forward result between the sweeps)
};

__device__ inline cplx ld_or_zero(const cplx* p, int64_t i, int64_t n) {
    return (i >= 0 && i < n) ? p[i] : mk(0.0, 0.0);
}

}  // namespace

__global__ void k_band_sweep(SweepArgs a) {
    __shared__ cplx slotX[2], slotA[2];
    if (a.active != nullptr && *a.active == 0) return;
    const int W = blockDim.x;
    const int t = threadIdx.x;
    const int64_t n = a.n;

    // ---------------- forward sweep with interleaved interchanges ----------------
    int64_t row = t;
    cplx val = ld_or_zero(a.u, row, n);
    int pj = a.ipiv[0];
    if (row == 0) slotA[0] = val;
    if (row == pj) slotX[0] = val;

    auto row_at = [&](int64_t r, int64_t jj) -> int64_t { return (r >= jj) ? r : r + W; };
    auto lval = [&](int64_t r, int64_t jj) -> cplx {
        if (jj >= n) return mk(0.0, 0.0);
        const int64_t d = row_at(r, jj) - jj;
        const int64_t km = min((int64_t)a.kl, n - 1 - jj);
        if (d < 1 || d > km) return mk(0.0, 0.0);
        return a.AB[(int64_t)(a.kv + d) + jj * a.ldab];
    };
    auto piv = [&](int64_t jj) -> int { return (jj < n) ? a.ipiv[jj] : -1; };

    cplx lring[PF], inring[PF];
    int pring[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        lring[q] = lval(row, q);
        pring[q] = piv(q + 1);
        inring[q] = ld_or_zero(a.u, row_at(row, q) + W, n);
    }

    for (int64_t j0 = 0; j0 < n; j0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int64_t j = j0 + q;
            if (j >= n) break;
            const cplx lj = lring[q];
            const int pj1 = pring[q];
            const cplx nin = inring[q];
            lring[q] = lval(row, j + PF);
            pring[q] = piv(j + PF + 1);
            inring[q] = ld_or_zero(a.u, row_at(row, j + PF) + W, n);
            __syncthreads();
            const cplx X = slotX[j & 1];
            const cplx A = slotA[j & 1];
            if (row == j) {
                a.y[j] = X;
                row += W;
                val = nin;
            } else {
                // the pivot row receives row j's old value; lj is zero outside the band
                val = fms((row == pj) ? A : val, lj, X);
            }
            if (row == j + 1) slotA[(j + 1) & 1] = val;
            if (row == pj1) slotX[(j + 1) & 1] = val;
            pj = pj1;
        }
    }
    __syncthreads();

    // ---------------- backward sweep ----------------
    // thread t owns rows i = t (mod W) in the window [j - W + 1, j]
    {
        const int64_t base = n - W;
        row = base + (((t - base) % W) + W) % W;
    }
    val = ld_or_zero(a.y, row, n);
    if (row == n - 1) slotA[(n - 1) & 1] = val;
    auto row_atb = [&](int64_t r, int64_t jj) -> int64_t { return (r <= jj) ? r : r - W; };
    auto uval = [&](int64_t r, int64_t jj) -> cplx {
        if (jj < 0) return mk(0.0, 0.0);
        const int64_t d = jj - row_atb(r, jj);
        const int64_t km = min((int64_t)a.kv, jj);
        if (d < 1 || d > km) return mk(0.0, 0.0);
        return a.AB[(int64_t)(a.kv - d) + jj * a.ldab];
    };
    auto dval = [&](int64_t jj) -> cplx { return (jj >= 0) ? a.AB[(int64_t)a.kv + jj * a.ldab] : mk(1.0, 0.0); };
    cplx dring[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int64_t jj = n - 1 - q;
        lring[q] = uval(row, jj);
        dring[q] = dval(jj);
        inring[q] = ld_or_zero(a.y, row_atb(row, jj) - W, n);
    }
    __syncthreads();

    for (int64_t j0 = n - 1; j0 >= 0; j0 -= PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int64_t j = j0 - q;
            if (j < 0) break;
            const cplx uj = lring[q];
            const cplx diag = dring[q];
            const cplx nz = inring[q];
            lring[q] = uval(row, j - PF);
            dring[q] = dval(j - PF);
            inring[q] = ld_or_zero(a.y, row_atb(row, j - PF) - W, n);
            __syncthreads();
            const cplx A = slotA[j & 1];
            const cplx xj = cdiv(A, diag);
            if (row == j) {
                a.y[j] = xj;
                row -= W;
                val = nz;
            } else {
                val = fms(val, uj, xj);
            }
            if (row == j - 1) slotA[(j - 1) & 1] = val;
        }
    }
}

// u = s * B x (B banded, or the identity when Bb == NULL); optionally xs = s * x.
// s = 1 / *hdiv if hdiv != NULL.  Skipped when *active == 0.
__global__ void k_prepare_input(int64_t n, const cplx* __restrict__ x, const cplx* __restrict__ Bb, int klb, int kub,
                                const double* hdiv, const int* active, cplx* __restrict__ u, cplx* __restrict__ xs) {
    if (active != nullptr && *active == 0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = (hdiv != nullptr) ? *hdiv : 1.0;
    // the normalised basis vector is w / h (a division, as written in the Arnoldi step)
    auto xsv = [&](int64_t c) -> cplx { cplx v = x[c]; return (hdiv != nullptr) ? mk(v.re / h, v.im / h) : v; };
    if (xs != nullptr) xs[i] = xsv(i);
    if (Bb == nullptr) {
        u[i] = xsv(i);
        return;
    }
    const int ldb = klb + kub + 1;
    cplx acc = mk(0.0, 0.0);
    for (int d = -klb; d <= kub; ++d) {
        const int64_t c = i + d;
        if (c < 0 || c >= n) continue;
        acc = fma_c(acc, Bb[(int64_t)(kub - d) + c * ldb], xsv(c));
    }
    u[i] = acc;
}

simm_status prepare_input(int64_t n, const cplx* x, const cplx* Bb, int klb, int kub, const double* hdiv,
                          const int* active, cplx* u, cplx* xs, hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_prepare_input, dim3(blocks), dim3(256), 0, st, n, x, Bb, klb, kub, hdiv, active, u, xs);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

int sweep_threads(int kl, int ku) {
    int W = 64;
    while (W < kl + ku + 2) W *= 2;
    return W;
}

simm_status band_sweep(int64_t n, int kl, int ku, const cplx* AB, const int* ipiv, const cplx* u, const int* active,
                       cplx* y, hipStream_t st) {
    SweepArgs a;
    a.n = n;
    a.kl = kl;
    a.kv = kl + ku;
    a.ldab = 2 * kl + ku + 1;
    a.AB = AB;
    a.ipiv = ipiv;
    a.u = u;
    a.active = active;
    a.y = y;
    const int W = sweep_threads(kl, ku);
    if (W > 1024) {
        set_error("band too wide for the sweep kernel (kl + ku + 2 > 1024)");
        return SIMM_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(k_band_sweep, dim3(1), dim3(W), 0, st, a);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
