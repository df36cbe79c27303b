// Partitioned application of the band LU factor: y = U^{-1} L^{-1} P u
// (the Cayley operator of Sec. 2, eq. (IMxb), is M x = U^{-1} L^{-1} P B x).
//
// A sweep over the n columns is a linear state machine: before column J of the
// forward sweep the rows still receiving updates are J .. J+kl-1 (kl values, the
// "state"), and before column J-1 of the backward sweep they are J-K .. J-1
// (K = effective upper bandwidth of U).  The columns are cut into P chunks of s
// columns.  For chunk c, with state t_c at its start and its input rows,
//     [y_c ; t_{c+1}] = [y0_c ; tau_c] + [Psi_c ; Phi_c] t_c,
// where (y0_c, tau_c) is the chunk's response to its input with a zero state and
// Psi_c, Phi_c its response to a unit state.  Per application:
//   1. all chunks in parallel: zero-state chunk sweeps -> y0_c, tau_c;
//   2. the chain t_{c+1} = tau_c + Phi_c t_c (short; P steps of a K x K product),
//      run by a few workgroups that meet at a device-scope barrier per step;
//   3. all rows in parallel: y_c = y0_c + Psi_c t_c.
// Psi_c and Phi_c depend only on the factor and are formed once per shift by the
// same chunk kernel run with unit states.  This is the partitioning idea of
// Polizzi and Sameh's SPIKE algorithm, applied to the triangular factors (the
// factorization itself is the ordinary band LU with partial pivoting).
//
// Chunk kernel: one workgroup per (chunk, state vector).  Thread t owns the rows
// i = t (mod W) of the active window and keeps their values in registers; per
// column step only the pivot row and row j cross threads, through a
// parity-indexed LDS slot and one LDS-only barrier.  Pivot indices, diagonals,
// chunk inputs and outputs are staged in LDS, so the only global loads inside the
// column loop are the factor entries, issued PF columns ahead into a register
// ring.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

constexpr int PF = 16;   // factor prefetch distance (columns)

__device__ inline cplx ldz(const cplx* p, int64_t i, int64_t n) { return (i >= 0 && i < n) ? p[i] : mk(0.0, 0.0); }

}  // namespace

// ---------------------------------------------------------------------------
// forward (L) chunk sweep
// ---------------------------------------------------------------------------
template <int MAXW>
__global__ __launch_bounds__(MAXW) void k_chunk_fwd(SpikeFwd a) {
    if (a.active != nullptr && *a.active == 0) return;
    extern __shared__ cplx sm[];
    __shared__ cplx slotX[2], slotA[2];
    const int W = blockDim.x;
    const int t = threadIdx.x;
    const int n = (int)a.n;
    const int kl = a.kl;
    const int c = blockIdx.x;
    const int r_unit = blockIdx.y;              // mode 1: which unit state
    const int J0 = c * (int)a.s;
    const int J1 = min(n, J0 + (int)a.s);
    const int len = J1 - J0;
    const int nin = len + kl;                   // input rows J0 .. J1+kl-1
    cplx* outb = sm;                            // len
    cplx* inb = sm + a.s;                       // nin
    int* piv = reinterpret_cast<int*>(sm + 2 * a.s + kl + 1);   // len + 1
    for (int q = t; q < len; q += W) piv[q] = a.ipiv[J0 + q];
    if (t == 0) piv[len] = -1;
    if (a.mode == 0) {
        for (int q = t; q < nin; q += W) inb[q] = (q < kl || J0 + q >= n) ? mk(0.0, 0.0) : a.u[J0 + q];
    }
    __syncthreads();

    // value entering the window for a row (state rows first, then chunk input)
    auto inval = [&](int row) -> cplx {
        const int q = row - J0;
        const bool in = (row < n && q < nin);
        if (a.mode == 0) return csel(in, inb[min(q, nin - 1)], mk(0.0, 0.0));
        return mk((in && q == r_unit) ? 1.0 : 0.0, 0.0);
    };
    // Factor entry for my row at step jj.  Every thread loads something every step
    // (out-of-band taps read the zero entry stored after the band), so the loads in
    // flight are the same on every path and the compiler's waits stay exact.
    const int64_t colstep = a.ldab - 1;         // (row, jj) -> kv + row + jj (ldab - 1)
    auto lidx = [&](int r, int jj) -> int64_t {
        const int rr = (r >= jj) ? r : r + W;
        const int d = rr - jj;
        const bool ok = jj < J1 && d >= 1 && d <= kl && rr < n;
        return ok ? (int64_t)(a.kv + rr) + (int64_t)jj * colstep : a.zidx;
    };
    int row = J0 + ((t - J0 % W) % W + W) % W;
    cplx val = inval(row);
    int pj = piv[0];
    if (row == J0) slotA[J0 & 1] = val;
    if (row == pj) slotX[J0 & 1] = val;
    cplx ring[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) ring[q] = a.AB[lidx(row, J0 + q)];
    lds_barrier();

    // One column step.  The ring slot is consumed before it is refilled (no
    // loop-carried register copies); memory operations sit outside branches.
    auto step = [&](int j, cplx& slot) {
        const int pj1 = piv[j + 1 - J0];
        const cplx X = slotX[j & 1];
        const cplx A = slotA[j & 1];
        const cplx upd = fms(csel(row == pj, A, val), slot, X);   // zero factor outside the band
        if (row == j) {
            outb[j - J0] = X;
            row += W;
            val = inval(row);
        } else {
            val = upd;
        }
        slot = a.AB[lidx(row, j + PF)];
        if (row == j + 1) slotA[(j + 1) & 1] = val;
        if (row == pj1) slotX[(j + 1) & 1] = val;
        pj = pj1;
        lds_barrier();
    };
    int j0 = J0;
    for (; j0 + PF <= J1; j0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) step(j0 + q, ring[q]);
    }
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (j0 + q < J1) step(j0 + q, ring[q]);

    // end state: rows J1 .. J1+kl-1
    const int qe = row - J1;
    if (qe >= 0 && qe < kl) {
        const cplx v = (row < n) ? val : mk(0.0, 0.0);
        if (a.mode == 0) a.tau[(int64_t)c * kl + qe] = v;
        else a.Phi[(int64_t)c * kl * kl + (int64_t)qe * kl + r_unit] = v;    // Phi_c(i, r) at [c][i][r]
    }
    __syncthreads();
    for (int q = t; q < len; q += W) {
        if (a.mode == 0) a.y[J0 + q] = outb[q];
        else a.Psi[(int64_t)(J0 + q) + (int64_t)r_unit * n] = outb[q];
    }
}

// ---------------------------------------------------------------------------
// backward (U) chunk sweep
// ---------------------------------------------------------------------------
template <int MAXW>
__global__ __launch_bounds__(MAXW) void k_chunk_bwd(SpikeBwd a) {
    if (a.active != nullptr && *a.active == 0) return;
    extern __shared__ cplx sm[];
    __shared__ cplx slotA[2];
    const int W = blockDim.x;
    const int t = threadIdx.x;
    const int n = (int)a.n;
    const int K = a.K;
    const int c = blockIdx.x;
    const int r_unit = blockIdx.y;
    const int J0 = c * (int)a.s;
    const int J1 = min(n, J0 + (int)a.s);
    const int len = J1 - J0;
    const int ib0 = J0 - W;                     // input rows [J0 - W, J1 - K)
    const int nib = len + W;
    cplx* outb = sm;                            // len
    cplx* dg = sm + a.s;                        // len diagonals
    cplx* inb = sm + 2 * a.s;                   // nib
    for (int q = t; q < len; q += W) dg[q] = a.AB[(int64_t)a.kvf + (int64_t)(J0 + q) * a.ldab];
    if (a.mode == 0) {
        for (int q = t; q < nib; q += W) {
            const int row = ib0 + q;
            inb[q] = (row >= 0 && row < J1 - K && row < n) ? a.z[row] : mk(0.0, 0.0);
        }
    }
    __syncthreads();

    auto inval = [&](int row) -> cplx {
        const bool state = row >= J1 - K;       // state rows: zero, or the unit vector
        if (a.mode == 0) return csel(row >= 0 && !state, inb[max(0, min(row - ib0, nib - 1))], mk(0.0, 0.0));
        return mk((row >= 0 && state && row - (J1 - K) == r_unit) ? 1.0 : 0.0, 0.0);
    };
    const int64_t colstep = a.ldab + 1;         // (row, jj) -> kvf - jj + row + jj ldab
    auto uidx = [&](int r, int jj) -> int64_t {
        const int rr = (r <= jj) ? r : r - W;
        const int d = jj - rr;
        const bool ok = jj >= J0 && d >= 1 && d <= K && rr >= 0;
        return ok ? (int64_t)(a.kvf + rr) + (int64_t)jj * colstep - 2 * (int64_t)jj : a.zidx;
    };
    const int base = J1 - W;
    int row = base + ((t - base % W) % W + W) % W;
    cplx val = inval(row);
    if (row == J1 - 1) slotA[(J1 - 1) & 1] = val;
    cplx ring[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) ring[q] = a.AB[uidx(row, J1 - 1 - q)];
    lds_barrier();

    auto step = [&](int j, cplx& slot) {
        const cplx A = slotA[j & 1];
        const cplx xj = cdiv(A, dg[j - J0]);
        const cplx upd = fms(val, slot, xj);
        if (row == j) {
            outb[j - J0] = xj;
            row -= W;
            val = inval(row);
        } else {
            val = upd;
        }
        slot = a.AB[uidx(row, j - PF)];
        if (row == j - 1) slotA[(j - 1) & 1] = val;
        lds_barrier();
    };
    int j0 = J1 - 1;
    for (; j0 - PF + 1 >= J0; j0 -= PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) step(j0 - q, ring[q]);
    }
#pragma unroll
    for (int q = 0; q < PF; ++q)
        if (j0 - q >= J0) step(j0 - q, ring[q]);

    // end state: rows J0 - K .. J0 - 1
    const int qe = row - (J0 - K);
    if (qe >= 0 && qe < K) {
        const cplx v = (row >= 0) ? val : mk(0.0, 0.0);
        if (a.mode == 0) a.tau[(int64_t)c * K + qe] = v;
        else a.Phi[(int64_t)c * K * K + (int64_t)qe * K + r_unit] = v;
    }
    __syncthreads();
    for (int q = t; q < len; q += W) {
        if (a.mode == 0) a.y[J0 + q] = outb[q];
        else a.Psi[(int64_t)(J0 + q) + (int64_t)r_unit * n] = outb[q];
    }
}

// ---------------------------------------------------------------------------
// chain over the chunk boundaries: t_{next} = tau_c + Phi_c t_c
// G workgroups own row slices of the state and meet at a device-scope barrier
// (monotone counter) after each step; a bounded spin turns a missing partner
// into an error flag instead of a hang.  Each thread keeps its part of the
// next step's Phi row in registers, loaded while the barrier is pending.
// ---------------------------------------------------------------------------
constexpr int CH_THREADS = 256;
constexpr int CH_PARTS = 16;                         // threads per state row
constexpr int CH_ROWS = CH_THREADS / CH_PARTS;       // state rows per workgroup

template <int MAXQ>
__global__ __launch_bounds__(CH_THREADS) void k_spike_chain(SpikeChain a) {
    if (a.active != nullptr && *a.active == 0) return;
    __shared__ cplx tcur[CH_PARTS * MAXQ];           // state, zero-padded
    const int K = a.K;
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int il = tid / CH_PARTS, part = tid % CH_PARTS;
    const int i = g * CH_ROWS + il;
    const int ic = min(i, K - 1);
    const int64_t KK = (int64_t)K * K;
    const int64_t c_first = a.forward ? 0 : a.P - 1;
    for (int r = tid; r < CH_PARTS * MAXQ; r += CH_THREADS) {
        const int64_t row = a.init_row0 + r;
        const cplx v = (r < K) ? ldz(a.init_src, row, a.n) : mk(0.0, 0.0);
        tcur[r] = v;
        if (g == 0 && r < K) a.t[c_first * K + r] = v;
    }
    cplx ph[MAXQ];
    auto load_phi = [&](int64_t c) {
        const cplx* prow = a.Phi + c * KK + (int64_t)ic * K;
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) ph[q] = prow[min(part + CH_PARTS * q, K - 1)];
    };
    if (a.P > 1) load_phi(c_first);
    __syncthreads();
    for (int64_t step = 0; step + 1 < a.P; ++step) {
        const int64_t c = a.forward ? step : a.P - 1 - step;
        const int64_t cn = a.forward ? c + 1 : c - 1;
        cplx acc = mk(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) acc = fma_c(acc, ph[q], tcur[part + CH_PARTS * q]);   // padded t is 0
        if (step + 2 < a.P) load_phi(a.forward ? c + 1 : c - 1);
#pragma unroll
        for (int m = CH_PARTS / 2; m >= 1; m >>= 1) {
            acc.re += __shfl_xor(acc.re, m, 64);
            acc.im += __shfl_xor(acc.im, m, 64);
        }
        if (part == 0 && i < K) a.t[cn * K + i] = a.tau[c * K + i] + acc;
        // device-scope barrier: every thread releases its stores, thread 0 arrives
        // and waits, every thread acquires
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_fetch_add(a.counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)(gridDim.x * (step + 1));
            long spins = 0;
            while (__hip_atomic_load(a.counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > 40000000L) {
                    atomicExch(a.err, 1);
                    break;
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int r = tid; r < K; r += CH_THREADS) tcur[r] = a.t[cn * K + r];
        __syncthreads();
    }
}

// y(j) += sum_r Psi(j, r) t_{c(j)}(r); the (at most two) state vectors a block
// needs are staged in LDS.
__global__ __launch_bounds__(256) void k_spike_correct(int64_t n, int K, int64_t s, const cplx* __restrict__ Psi,
                                                       const cplx* __restrict__ t, cplx* __restrict__ y,
                                                       const int* active) {
    if (active != nullptr && *active == 0) return;
    extern __shared__ cplx ts[];                     // 2 K
    const int64_t jb = (int64_t)blockIdx.x * blockDim.x;
    const int64_t cb = jb / s;
    const int64_t ce = min(n - 1, jb + (int64_t)blockDim.x - 1) / s;
    for (int r = threadIdx.x; r < K; r += blockDim.x) {
        ts[r] = t[cb * K + r];
        ts[K + r] = t[ce * K + r];
    }
    __syncthreads();
    const int64_t j = jb + threadIdx.x;
    if (j >= n) return;
    const cplx* tc = ts + ((j / s == cb) ? 0 : K);
    cplx acc = y[j];
    const cplx* pr = Psi + j;
    int r = 0;
    for (; r + 8 <= K; r += 8) {
        cplx v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pr[(int64_t)(r + u) * n];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma_c(acc, v[u], tc[r + u]);
    }
    for (; r < K; ++r) acc = fma_c(acc, pr[(int64_t)r * n], tc[r]);
    y[j] = acc;
}

__global__ void k_fill_u32(unsigned* p, int count, unsigned v) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = v;
}

// max_j (ipiv[j] - j)
__global__ void k_max_jump(int64_t n, const int* ipiv, int* out) {
    __shared__ int red[256];
    int best = 0;
    for (int64_t j = threadIdx.x; j < n; j += 256) best = max(best, (int)(ipiv[j] - j));
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

namespace {

int pow2_at_least(int v) {
    int w = 64;
    while (w < v) w *= 2;
    return w;
}

template <typename Args>
simm_status launch_fwd(const Args& a, int64_t P, int nrhs, int W, size_t lds, hipStream_t st) {
    if (W <= 256) hipLaunchKernelGGL(k_chunk_fwd<256>, dim3((unsigned)P, nrhs), dim3(W), lds, st, a);
    else if (W <= 512) hipLaunchKernelGGL(k_chunk_fwd<512>, dim3((unsigned)P, nrhs), dim3(W), lds, st, a);
    else hipLaunchKernelGGL(k_chunk_fwd<1024>, dim3((unsigned)P, nrhs), dim3(W), lds, st, a);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}
template <typename Args>
simm_status launch_bwd(const Args& a, int64_t P, int nrhs, int W, size_t lds, hipStream_t st) {
    if (W <= 256) hipLaunchKernelGGL(k_chunk_bwd<256>, dim3((unsigned)P, nrhs), dim3(W), lds, st, a);
    else if (W <= 512) hipLaunchKernelGGL(k_chunk_bwd<512>, dim3((unsigned)P, nrhs), dim3(W), lds, st, a);
    else hipLaunchKernelGGL(k_chunk_bwd<1024>, dim3((unsigned)P, nrhs), dim3(W), lds, st, a);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

size_t fwd_lds(int64_t s, int kl) { return sizeof(cplx) * (size_t)(2 * s + kl + 1) + sizeof(int) * (size_t)(s + 2) + 64; }
size_t bwd_lds(int64_t s, int W) { return sizeof(cplx) * (size_t)(3 * s + W) + 64; }

}  // namespace

int64_t spike_chunk_len(int64_t n, int kl, int K) {
    int64_t s = 0;
    if (const char* e = getenv("SIMM_SPIKE_CHUNK")) s = atoll(e);
    if (s <= 0) s = std::max<int64_t>(256, (n + 47) / 48);
    s = std::min<int64_t>(s, 2048);
    s = std::max<int64_t>(s, std::max(kl, K) + 1);
    return std::min<int64_t>(s, n);
}

simm_status spike_prepare(SpikeFactor& f, hipStream_t st) {
    // effective upper bandwidth of U: ku plus the largest interchange distance
    int* d_jump = nullptr;
    SIMM_HIP_TRY(hipMallocAsync((void**)&d_jump, sizeof(int), st));
    hipLaunchKernelGGL(k_max_jump, dim3(1), dim3(256), 0, st, f.n, (const int*)f.ipiv, d_jump);
    int jump = 0;
    SIMM_HIP_TRY(hipMemcpyAsync(&jump, d_jump, sizeof(int), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    SIMM_HIP_TRY(hipFreeAsync(d_jump, st));
    f.K = (int)std::min<int64_t>(std::min<int64_t>(f.kl + f.ku, f.ku + std::max(0, jump)), f.n - 1);
    f.K = std::max(f.K, 0);
    f.klx = (int)std::min<int64_t>(f.kl, f.n - 1);
    f.s = spike_chunk_len(f.n, f.klx, f.K);
    f.P = (f.n + f.s - 1) / f.s;
    if (f.n > (int64_t)1 << 30) {
        set_error("order above 2^30 is not supported by the partitioned sweeps");
        return SIMM_EUNSUPPORTED;
    }
    f.Wf = pow2_at_least(f.klx + 2);
    f.Wb = pow2_at_least(f.K + 2);
    if (f.Wf > 1024 || f.Wb > 1024) {
        set_error("band too wide for the partitioned sweeps (bandwidth + 2 > 1024)");
        return SIMM_EUNSUPPORTED;
    }
    const int kl = std::max(f.klx, 1), K = std::max(f.K, 1);
    const size_t bytes = sizeof(cplx) * ((size_t)f.n * kl + (size_t)f.P * kl * kl + (size_t)f.n * K +
                                         (size_t)f.P * K * K + (size_t)f.P * kl * 2 + (size_t)f.P * K * 2 +
                                         (size_t)f.n) + 1024 + 8 * 256;
    SIMM_HIP_TRY(hipMalloc(&f.mem, bytes));
    char* p = reinterpret_cast<char*>(f.mem);
    auto take = [&](size_t b) {
        char* r = p;
        p += (b + 255) & ~(size_t)255;
        return r;
    };
    f.PsiL = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.n * kl));
    f.PhiL = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.P * kl * kl));
    f.PsiU = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.n * K));
    f.PhiU = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.P * K * K));
    f.tauL = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.P * kl));
    f.tL = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.P * kl));
    f.tauU = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.P * K));
    f.tU = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.P * K));
    f.z = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)f.n));
    f.counter = reinterpret_cast<unsigned*>(take(64));
    f.err = reinterpret_cast<int*>(take(64));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(f.err), 1, 0u);
    // unit-state responses Psi, Phi
    if (f.klx > 0) {
        SpikeFwd a{};
        a.n = f.n;
        a.kl = f.klx;
        a.kv = f.kl + f.ku;
        a.ldab = 2 * f.kl + f.ku + 1;
        a.AB = f.AB;
        a.ipiv = f.ipiv;
        a.s = f.s;
        a.mode = 1;
        a.zidx = (int64_t)(2 * f.kl + f.ku + 1) * f.n;
        a.Psi = f.PsiL;
        a.Phi = f.PhiL;
        SIMM_TRY(launch_fwd(a, f.P, f.klx, f.Wf, fwd_lds(f.s, f.klx), st));
    }
    if (f.K > 0) {
        SpikeBwd b{};
        b.n = f.n;
        b.K = f.K;
        b.kvf = f.kl + f.ku;
        b.ldab = 2 * f.kl + f.ku + 1;
        b.AB = f.AB;
        b.s = f.s;
        b.mode = 1;
        b.zidx = (int64_t)(2 * f.kl + f.ku + 1) * f.n;
        b.Psi = f.PsiU;
        b.Phi = f.PhiU;
        SIMM_TRY(launch_bwd(b, f.P, f.K, f.Wb, bwd_lds(f.s, f.Wb), st));
    }
    return SIMM_OK;
}

void spike_release(SpikeFactor& f) {
    (void)hipFree(f.mem);
    f.mem = nullptr;
}

static simm_status run_chain(const SpikeFactor& f, bool forward, int K, const cplx* Phi, const cplx* tau, cplx* tstate,
                             const cplx* init_src, int64_t init_row0, const int* active, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, f.counter, 1, 0u);
    SpikeChain c{};
    c.n = f.n;
    c.K = K;
    c.P = f.P;
    c.forward = forward ? 1 : 0;
    c.Phi = Phi;
    c.tau = tau;
    c.t = tstate;
    c.init_src = init_src;
    c.init_row0 = init_row0;
    c.counter = f.counter;
    c.err = f.err;
    c.active = active;
    const int G = (K + CH_ROWS - 1) / CH_ROWS;
    if (K <= 16 * CH_PARTS) hipLaunchKernelGGL(k_spike_chain<16>, dim3(G), dim3(CH_THREADS), 0, st, c);
    else if (K <= 32 * CH_PARTS) hipLaunchKernelGGL(k_spike_chain<32>, dim3(G), dim3(CH_THREADS), 0, st, c);
    else hipLaunchKernelGGL(k_spike_chain<64>, dim3(G), dim3(CH_THREADS), 0, st, c);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status spike_apply(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st) {
    const unsigned blocks = (unsigned)((f.n + 255) / 256);
    // forward: z = L^{-1} P u
    cplx* z = f.z;
    if (f.klx > 0) {
        SpikeFwd a{};
        a.n = f.n;
        a.kl = f.klx;
        a.kv = f.kl + f.ku;
        a.ldab = 2 * f.kl + f.ku + 1;
        a.AB = f.AB;
        a.ipiv = f.ipiv;
        a.s = f.s;
        a.mode = 0;
        a.zidx = (int64_t)(2 * f.kl + f.ku + 1) * f.n;
        a.u = u;
        a.y = z;
        a.tau = f.tauL;
        a.active = active;
        SIMM_TRY(launch_fwd(a, f.P, 1, f.Wf, fwd_lds(f.s, f.klx), st));
        SIMM_TRY(run_chain(f, true, f.klx, f.PhiL, f.tauL, f.tL, u, 0, active, st));
        hipLaunchKernelGGL(k_spike_correct, dim3(blocks), dim3(256), sizeof(cplx) * 2 * f.klx, st, f.n, f.klx, f.s,
                           (const cplx*)f.PsiL, (const cplx*)f.tL, z, active);
    } else {
        SIMM_HIP_TRY(hipMemcpyAsync(z, u, sizeof(cplx) * f.n, hipMemcpyDeviceToDevice, st));
    }
    // backward: y = U^{-1} z
    SpikeBwd b{};
    b.n = f.n;
    b.K = f.K;
    b.kvf = f.kl + f.ku;
    b.ldab = 2 * f.kl + f.ku + 1;
    b.AB = f.AB;
    b.s = f.s;
    b.mode = 0;
    b.zidx = (int64_t)(2 * f.kl + f.ku + 1) * f.n;
    b.z = z;
    b.y = y;
    b.tau = f.tauU;
    b.active = active;
    SIMM_TRY(launch_bwd(b, f.P, 1, f.Wb, bwd_lds(f.s, f.Wb), st));
    if (f.K > 0) {
        SIMM_TRY(run_chain(f, false, f.K, f.PhiU, f.tauU, f.tU, z, f.n - f.K, active, st));
        hipLaunchKernelGGL(k_spike_correct, dim3(blocks), dim3(256), sizeof(cplx) * 2 * f.K, st, f.n, f.K, f.s,
                           (const cplx*)f.PsiU, (const cplx*)f.tU, y, active);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

int64_t spike_bytes_per_apply(const SpikeFactor& f) {
    // algorithmic bytes: each stored factor entry within the effective band read once,
    // input read once, output written once
    int64_t lower = 0, upper = 0;
    for (int64_t j = 0; j < f.n; ++j) {
        lower += std::min<int64_t>(f.kl, f.n - 1 - j);
        upper += std::min<int64_t>(f.K, j) + 1;
    }
    return 16 * (lower + upper + 2 * f.n);
}

}  // namespace simm
