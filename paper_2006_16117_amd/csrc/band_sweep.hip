// Input of the sweeps: u = B x for the Cayley operator M = (A - sigma B)^{-1} B of
// Sec. 2, eq. (IMxb) (and the normalised basis vector x / h when requested).
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

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

}  // namespace simm
