// FP64-residual iterative refinement of solves with an FP32 band factor (mixed
// precision).  The Cayley transform of Sec. 2 needs y = (A - sigma B)^{-1} u for every
// application of M (eq. (IMxb)); with the factor L U ~ P (A - sigma B) held in FP32,
//     x_0 = U^{-1} L^{-1} P u,   r_k = u - (A - sigma B) x_k  (FP64, from the FP64 bands),
//     x_{k+1} = x_k + U^{-1} L^{-1} P r_k,
// until the normwise backward error
//     eta_k = ||r_k||_inf / (||A - sigma B||_inf ||x_k||_inf + ||u||_inf)
// is at most the tolerance.  Every step is decided on the device (a flag that the
// next kernels read), so an application never waits for the host; a step that is not
// needed returns at once.  If the tolerance is not met within the allowed steps an
// error flag is raised and the shift is rebuilt with an FP64 factor by the caller.
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

// non-negative doubles order like their bit patterns
__device__ inline void atomic_max_nonneg(unsigned long long* p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}
__device__ inline double wave_max64(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

}  // namespace

// r = u - (A - sigma B) x, row by row, and the infinity norms of r, x and u
// (norms[0..2], as the bit patterns of non-negative doubles).  Skipped when *gate == 0.
// A wavefront takes 64 consecutive rows and walks the columns that meet them: at
// column j its lanes read the entries (i, j) of their rows, which are consecutive in
// band storage (one coalesced load; x_j is the same for every lane).  Each row still
// accumulates its entries in ascending column order.
__global__ __launch_bounds__(256) void k_band_resid(int64_t n, const cplx* __restrict__ A, int kla, int kua,
                                                    const cplx* __restrict__ B, int klb, int kub, cplx sigma,
                                                    const cplx* __restrict__ u, const cplx* __restrict__ x,
                                                    cplx* __restrict__ r, unsigned long long* norms, const int* gate) {
    if (*gate == 0) return;
    const int64_t r0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);   // first row of this wavefront
    const int64_t i = r0 + (threadIdx.x & 63);
    double nr = 0.0, nx = 0.0, nu = 0.0;
    if (r0 < n) {
        const int lda = kla + kua + 1;
        const bool row = i < n;
        cplx acc = row ? u[i] : mk(0.0, 0.0);
        const int64_t jlo = max((int64_t)0, r0 - kla), jhi = min(n - 1, r0 + 63 + kua);
#pragma unroll 4
        for (int64_t j = jlo; j <= jhi; ++j) {
            const cplx xj = x[j];
            const int64_t d = j - i;
            if (row && d >= -kla && d <= kua) acc = fms(acc, A[(kua - d) + j * lda], xj);
        }
        if (row && B != nullptr) {
            const int ldb = klb + kub + 1;
            const int elo = (int)max((int64_t)-klb, -i), ehi = (int)min((int64_t)kub, n - 1 - i);
            cplx bx = mk(0.0, 0.0);
            for (int d = elo; d <= ehi; ++d) bx = fma_c(bx, B[(int64_t)(kub - d) + (i + d) * ldb], x[i + d]);
            acc = fma_c(acc, sigma, bx);
        } else if (row) {
            acc = fma_c(acc, sigma, x[i]);
        }
        if (row) {
            r[i] = acc;
            nr = cabs(acc);
            nx = cabs(x[i]);
            nu = cabs(u[i]);
        }
    }
    nr = wave_max64(nr);
    nx = wave_max64(nx);
    nu = wave_max64(nu);
    if ((threadIdx.x & 63) == 0) {
        atomic_max_nonneg(norms + 0, nr);
        atomic_max_nonneg(norms + 1, nx);
        atomic_max_nonneg(norms + 2, nu);
    }
}

// ||A - sigma B||_inf into norms[0] (bit pattern).  Rows and columns are walked as in
// k_band_resid (64 rows per wavefront, coalesced loads, each row in ascending column
// order).
__global__ __launch_bounds__(256) void k_band_rownorm(int64_t n, const cplx* __restrict__ A, int kla, int kua,
                                                      const cplx* __restrict__ B, int klb, int kub, cplx sigma,
                                                      unsigned long long* out) {
    const int64_t r0 = (int64_t)blockIdx.x * 256 + (threadIdx.x & ~63);   // first row of this wavefront
    const int64_t i = r0 + (threadIdx.x & 63);
    double s = 0.0;
    if (r0 < n) {
        const int lda = kla + kua + 1, ldb = klb + kub + 1;
        const int lo = -max(kla, B ? klb : 0), hi = max(kua, B ? kub : 0);
        const int64_t jlo = max((int64_t)0, r0 + lo), jhi = min(n - 1, r0 + 63 + hi);
        for (int64_t j = jlo; j <= jhi; ++j) {
            const int64_t dd = j - i;
            if (i >= n || dd < lo || dd > hi) continue;
            const int d = (int)dd;
            cplx c = (d >= -kla && d <= kua) ? A[(int64_t)(kua - d) + j * lda] : mk(0.0, 0.0);
            if (B != nullptr) {
                if (d >= -klb && d <= kub) c = fms(c, sigma, B[(int64_t)(kub - d) + j * ldb]);
            } else if (d == 0) {
                c = c - sigma;
            }
            s += cabs(c);
        }
    }
    s = wave_max64(s);
    if ((threadIdx.x & 63) == 0) atomic_max_nonneg(out, s);
}

// state[0] = refinement active (starts as *active, or 1), norms cleared
__global__ void k_refine_start(const int* active, RefineState st) {
    st.flags[0] = (active == nullptr || *active != 0) ? 1 : 0;
    st.norms[0] = st.norms[1] = st.norms[2] = 0ull;
}

// After a residual: converged (eta <= tol) ends the refinement; otherwise one more
// correction, or, after the last allowed one, the error flag.  Clears the norms.
__global__ void k_refine_check(RefineState st, double cnorm, double tol, int last) {
    if (st.flags[0] == 0) return;
    const double nr = __longlong_as_double((long long)st.norms[0]);
    const double nx = __longlong_as_double((long long)st.norms[1]);
    const double nu = __longlong_as_double((long long)st.norms[2]);
    st.norms[0] = st.norms[1] = st.norms[2] = 0ull;
    const double den = cnorm * nx + nu;
    const double eta = den > 0.0 ? nr / den : 0.0;
    if (eta <= tol) {
        st.flags[0] = 0;
        st.stats[0] += 1;                           // applications
        if (eta > __longlong_as_double((long long)st.norms[3])) st.norms[3] = (unsigned long long)__double_as_longlong(eta);
    } else if (last) {
        st.flags[0] = 0;
        st.flags[1] = 1;                            // tolerance not reached
        st.stats[0] += 1;
        if (eta > __longlong_as_double((long long)st.norms[3])) st.norms[3] = (unsigned long long)__double_as_longlong(eta);
    } else {
        st.stats[1] += 1;                           // corrections
    }
}

__global__ __launch_bounds__(256) void k_axpy_gated(int64_t n, cplx* __restrict__ x, const cplx* __restrict__ d,
                                                    const int* gate) {
    if (*gate == 0) return;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = x[i] + d[i];
}

simm_status band_inf_norm(int64_t n, const cplx* A, int kla, int kua, const cplx* B, int klb, int kub, cplx sigma,
                          unsigned long long* out, double* host, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, st, out, 1);
    hipLaunchKernelGGL(k_band_rownorm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, A, kla, kua, B, klb, kub,
                       sigma, out);
    unsigned long long bits = 0;
    SIMM_HIP_TRY(hipMemcpyAsync(&bits, out, sizeof(bits), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(host, &bits, sizeof(double));
    return SIMM_OK;
}

// u_i = 1 + ((i mod 7) - 3) / 4 + i ((i mod 5) - 2) / 3: a fixed right-hand side with no
// zero entries and no structure aligned with a block partition
__global__ __launch_bounds__(256) void k_probe_rhs(int64_t n, cplx* __restrict__ u) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) u[i] = mk(1.0 + (double)((i % 7) - 3) / 4.0, (double)((i % 5) - 2) / 3.0);
}

simm_status solve_backward_error(const SpikeFactor& f, const RefinePencil& pen, double* eta, hipStream_t st) {
    const int64_t n = f.n;
    const int64_t n16 = (n + 15) / 16 * 16;
    void* mem = nullptr;
    SIMM_HIP_TRY(device_malloc_async(&mem, sizeof(cplx) * 3 * (size_t)n16 + 256, st));
    struct Free {
        void* q;
        hipStream_t st;
        ~Free() { (void)hipFreeAsync(q, st); }
    } fr{mem, st};
    cplx* u = reinterpret_cast<cplx*>(mem);
    cplx* x = u + n16;
    cplx* r = x + n16;
    unsigned long long* norms = reinterpret_cast<unsigned long long*>(r + n16);
    int* gate = reinterpret_cast<int*>(norms + 4);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_probe_rhs, dim3(blocks), dim3(256), 0, st, n, u);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, norms, 4);
    const int one = 1;
    SIMM_HIP_TRY(hipMemcpyAsync(gate, &one, sizeof(int), hipMemcpyHostToDevice, st));
    ChainSlots slots;   // released (after a synchronize) when this returns
    SIMM_TRY(slots.acquire(spike_chain_weight(f), st));
    SIMM_TRY(spike_apply(f, u, x, nullptr, st));
    hipLaunchKernelGGL(k_band_resid, dim3(blocks), dim3(256), 0, st, n, pen.A, pen.kla, pen.kua, pen.B, pen.klb,
                       pen.kub, pen.sigma, (const cplx*)u, (const cplx*)x, r, norms, (const int*)gate);
    SIMM_HIP_TRY(hipGetLastError());
    unsigned long long nb[3] = {0, 0, 0};
    SIMM_HIP_TRY(hipMemcpyAsync(nb, norms, sizeof(nb), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    double v[3];
    std::memcpy(v, nb, sizeof(v));
    const double den = pen.cnorm * v[1] + v[2];
    *eta = den > 0.0 ? v[0] / den : 0.0;
    if (!std::isfinite(v[0]) || !std::isfinite(v[1])) *eta = INFINITY;
    return SIMM_OK;
}

simm_status refine_apply(const SpikeFactor& f, const RefinePencil& pen, const RefineState& rs, const cplx* u, cplx* y,
                         const int* active, hipStream_t st) {
    const int64_t n = f.n;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    const int* gate = rs.flags;
    hipLaunchKernelGGL(k_refine_start, dim3(1), dim3(1), 0, st, active, rs);
    SIMM_TRY(spike_apply(f, u, y, active, st));
    for (int k = 0; k <= kRefineMaxSteps; ++k) {
        hipLaunchKernelGGL(k_band_resid, dim3(blocks), dim3(256), 0, st, n, pen.A, pen.kla, pen.kua, pen.B, pen.klb,
                           pen.kub, pen.sigma, u, (const cplx*)y, rs.r, rs.norms, gate);
        hipLaunchKernelGGL(k_refine_check, dim3(1), dim3(1), 0, st, rs, pen.cnorm, kRefineTol,
                           k == kRefineMaxSteps ? 1 : 0);
        if (k == kRefineMaxSteps) break;
        SIMM_TRY(spike_apply(f, rs.r, rs.d, gate, st));
        hipLaunchKernelGGL(k_axpy_gated, dim3(blocks), dim3(256), 0, st, n, y, (const cplx*)rs.d, gate);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
