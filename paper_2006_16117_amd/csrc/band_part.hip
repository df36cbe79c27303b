// Partitioned factorization of the shifted band (gfx950).
//
// The Cayley transform of Sec. 2 needs one factorization of C = A - sigma B per shift;
// a whole-matrix band LU is a chain of n/16 dependent panel steps.  Here C is split as
// C = D + E, D block diagonal (diagonal blocks D_j of bs columns, the last one shorter)
// and E the couplings between neighbouring blocks, in the divide-and-conquer form of the
// SPIKE algorithm (Polizzi and Sameh):
//   * every D_j is factored with partial pivoting inside the block, all blocks in the
//     same launches (the band LU in its block-diagonal mode), so a factor takes bs/16
//     panel steps instead of n/16;
//   * the spikes V = D^{-1} E_up, W = D^{-1} E_low: with boundary q_p = (p+1) bs, column
//     k of V holds, in the rows of block p, D_p^{-1} times the coupling of block p to
//     x[q_p + k] (k < ku); column k of W holds, in the rows of block p+1, D_{p+1}^{-1}
//     times the coupling of block p+1 to x[q_p - kl + k] (k < kl);
//   * the reduced system: with t_p = x[q_p .. q_p + ku) and b_p = x[q_p - kl .. q_p), the
//     rows of x = g - V t - W b at the tips give, per boundary p,
//         b_p + V(b rows) t_p + W(b rows) b_{p-1} = g(b rows)
//         t_p + W(t rows) b_p + V(t rows) t_{p+1} = g(t rows),
//     a band system R of order nr = (nbk - 1)(kl + ku) with lower bandwidth 2 kl + ku - 1
//     and upper kl + 2 ku - 1; R is factored by the band LU and inverted (nr <= 2048);
//   * a solve C y = u is g = D^{-1} u (the partitioned sweeps of D's factor), z = R^{-1}
//     tips(g), and y_i = g_i - sum_k V[i,k] t[k] - sum_k W[i,k] b[k] with the tips of the
//     boundaries of row i's block.
// Pivoting never crosses a block boundary, so the caller checks the backward error of a
// solve and factors the whole matrix instead when it is not small.
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace simm {

int64_t part_block_len(int64_t n, int kl, int ku) {
    const int w = kl + ku;
    if (kl < 1 || ku < 1) return 0;
    // the reduced system's band LU: its lower bandwidth within the LU kernel's reach
    if (lu_panel_width(2 * kl + ku - 1) == 0) return 0;
    int64_t bs = -1;
    if (const char* e = getenv("SIMM_LU_PART")) bs = atoll(e);   // 0: never; > 0: this block length
    if (bs == 0) return 0;
    // each block holds both tips of its boundaries, and a 256-row workgroup of the
    // correction spans at most two blocks
    const int64_t bmin = std::max<int64_t>(256, (2 * (int64_t)w + 15) / 16 * 16);
    if (bs > 0) {
        bs = std::max<int64_t>((bs + 15) / 16 * 16, bmin);
    } else {
        // as many blocks as keep the reduced order within kPartMaxReduced, each of at
        // least max(1024, 4 (kl + ku)) rows
        const int64_t nb_max = 1 + kPartMaxReduced / w;
        const int64_t nb = std::min<int64_t>(nb_max, n / std::max<int64_t>(1024, 4 * (int64_t)w));
        if (nb < 2) return 0;
        bs = std::max<int64_t>(((n + nb - 1) / nb + 15) / 16 * 16, bmin);
    }
    // the last block holds at least kl + ku rows
    for (int it = 0; it < 4096 && bs < n; ++it) {
        const int64_t nbk = (n + bs - 1) / bs;
        if (n - (nbk - 1) * bs >= w) break;
        bs += 16;
    }
    if (bs >= n) return 0;
    const int64_t nbk = (n + bs - 1) / bs;
    if ((nbk - 1) * (int64_t)w > kPartMaxReduced) return 0;
    return bs;
}

size_t part_cpl_elems(int64_t n, int kl, int ku, int64_t bs) {
    const int64_t nbk = (n + bs - 1) / bs;
    return (size_t)(nbk - 1) * ((size_t)ku * ku + (size_t)kl * kl);
}

namespace {

// One workgroup per boundary q = (p+1) bs: the coupling entries C(q - ku + i, q + k)
// (k <= i) and C(q + i, q - kl + k) (i <= k) out of the band, zeroed there.
template <typename CT>
__global__ __launch_bounds__(256) void k_part_cut(int64_t n, int kl, int ku, CT* __restrict__ AB, int64_t bs,
                                                  cplx* __restrict__ cpl) {
    const int p = blockIdx.x;
    const int64_t q = (int64_t)(p + 1) * bs;
    const int kv = kl + ku, ldab = 2 * kl + ku + 1;
    cplx* cu = cpl + (size_t)p * ((size_t)ku * ku + (size_t)kl * kl);
    cplx* cl = cu + (size_t)ku * ku;
    for (int e = threadIdx.x; e < ku * ku + kl * kl; e += blockDim.x) {
        int64_t row, col;
        bool valid;
        cplx* dst;
        if (e < ku * ku) {
            const int i = e % ku, k = e / ku;
            row = q - ku + i;
            col = q + k;
            valid = k <= i && col < n;
            dst = cu + e;
        } else {
            const int e2 = e - ku * ku;
            const int i = e2 % kl, k = e2 / kl;
            row = q + i;
            col = q - kl + k;
            valid = i <= k && row < n;
            dst = cl + e2;
        }
        cplx v = mk(0.0, 0.0);
        if (valid) {
            CT* at = AB + (int64_t)(kv + row - col) + col * ldab;
            v = widen(*at);
            *at = narrow<CT>(mk(0.0, 0.0));
        }
        *dst = v;
    }
}

// Right-hand side of spike column k: the upper couplings (which = 0, rows q_p - ku ..
// q_p - 1 of block p) or the lower ones (which = 1, rows q_p .. q_p + kl - 1 of block
// p+1), zero elsewhere; all n16 rows written.
__global__ __launch_bounds__(256) void k_part_rhs(int64_t n, int64_t n16, int kl, int ku, int64_t bs, int64_t nbk,
                                                  const cplx* __restrict__ cpl, int which, int k,
                                                  cplx* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n16) return;
    cplx v = mk(0.0, 0.0);
    if (i < n) {
        const int64_t j = i / bs;
        const size_t per = (size_t)ku * ku + (size_t)kl * kl;
        if (which == 0) {
            const int64_t q = (j + 1) * bs;
            if (j <= nbk - 2 && i >= q - ku) v = cpl[(size_t)j * per + (size_t)(i - (q - ku)) + (size_t)k * ku];
        } else {
            const int64_t q = j * bs;
            if (j >= 1 && i < q + kl) v = cpl[(size_t)(j - 1) * per + (size_t)ku * ku + (size_t)(i - q) + (size_t)k * kl];
        }
    }
    out[i] = v;
}

// Global row of reduced unknown c: b_p (r < kl) or t_p (r >= kl).
__device__ inline int64_t tip_row(int64_t c, int kl, int ku, int64_t bs) {
    const int w = kl + ku;
    const int64_t p = c / w;
    const int r = (int)(c - p * w);
    const int64_t q = (p + 1) * bs;
    return r < kl ? q - kl + r : q + (r - kl);
}

// The reduced band system (LAPACK band-LU layout, ldab = 2 klr + kur + 1; zeroed
// before), one thread per reduced row.
__global__ __launch_bounds__(256) void k_part_reduced(int64_t nr, int kl, int ku, int64_t bs, int64_t nbk,
                                                      int64_t n16, const cplx* __restrict__ V,
                                                      const cplx* __restrict__ W, cplx* __restrict__ ABr, int klr,
                                                      int kur) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nr) return;
    const int w = kl + ku;
    const int kvr = klr + kur, ldr = 2 * klr + kur + 1;
    const int64_t p = i / w;
    const int r = (int)(i - p * w);
    const int64_t gi = tip_row(i, kl, ku, bs);
    auto put = [&](int64_t col, cplx v) { ABr[(int64_t)(kvr + i - col) + col * ldr] = v; };
    put(i, mk(1.0, 0.0));
    if (r < kl) {
        for (int k = 0; k < ku; ++k) put(p * w + kl + k, V[gi + (int64_t)k * n16]);
        if (p >= 1)
            for (int k = 0; k < kl; ++k) put((p - 1) * w + k, W[gi + (int64_t)k * n16]);
    } else {
        for (int k = 0; k < kl; ++k) put(p * w + k, W[gi + (int64_t)k * n16]);
        if (p + 1 <= nbk - 2)
            for (int k = 0; k < ku; ++k) put((p + 1) * w + kl + k, V[gi + (int64_t)k * n16]);
    }
}

// Column c of R^{-1}: R y = e_c with R's band LU (interchanges and eliminations column
// by column as the factor stores them, then the upper triangular band solve), y in LDS;
// written as column c of the row-major inverse.
__global__ __launch_bounds__(256) void k_part_inverse(int64_t nr, int klr, int kur, const cplx* __restrict__ ABr,
                                                      const int* __restrict__ ipiv, cplx* __restrict__ Rinv) {
    extern __shared__ double2 ysm[];
    cplx* y = reinterpret_cast<cplx*>(ysm);
    const int64_t c = blockIdx.x;
    const int kvr = klr + kur, ldr = 2 * klr + kur + 1;
    for (int64_t i = threadIdx.x; i < nr; i += blockDim.x) y[i] = mk(i == c ? 1.0 : 0.0, 0.0);
    __syncthreads();
    for (int64_t j = 0; j < nr; ++j) {
        const int64_t pj = ipiv[j];
        if (threadIdx.x == 0 && pj != j) {
            const cplx t = y[j];
            y[j] = y[pj];
            y[pj] = t;
        }
        __syncthreads();
        const cplx yj = y[j];
        const int km = (int)std::min<int64_t>(klr, nr - 1 - j);
        for (int t = threadIdx.x; t < km; t += blockDim.x)
            y[j + 1 + t] = fms(y[j + 1 + t], ABr[(int64_t)(kvr + 1 + t) + j * ldr], yj);
        __syncthreads();
    }
    for (int64_t j = nr - 1; j >= 0; --j) {
        if (threadIdx.x == 0) y[j] = cdiv(y[j], ABr[(int64_t)kvr + j * ldr]);
        __syncthreads();
        const cplx yj = y[j];
        const int ku_j = (int)std::min<int64_t>(kvr, j);
        for (int t = threadIdx.x; t < ku_j; t += blockDim.x)
            y[j - 1 - t] = fms(y[j - 1 - t], ABr[(int64_t)(kvr - 1 - t) + j * ldr], yj);
        __syncthreads();
    }
    for (int64_t i = threadIdx.x; i < nr; i += blockDim.x) Rinv[i * nr + c] = y[i];
}

// z_i = sum_c Rinv[i, c] g[tip(c)] for NR right-hand sides (g + r ldg -> z + r ldz): one
// wavefront per reduced row, four accumulators per lane and column (a column's
// operations are those of NR = 1).
template <int NR>
__global__ __launch_bounds__(256) void k_part_tips(int64_t nr, int kl, int ku, int64_t bs,
                                                   const cplx* __restrict__ Rinv, const cplx* __restrict__ g,
                                                   int64_t ldg, cplx* __restrict__ z, int64_t ldz,
                                                   const int* active) {
    if (active && *active == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nr) return;
    const cplx* row = Rinv + i * nr;
    cplx acc[NR][4];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[r][u] = mk(0.0, 0.0);
    int64_t c = lane;
    for (; c + 3 * 64 < nr; c += 4 * 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const cplx rv = row[c + u * 64];
            const int64_t tr = tip_row(c + u * 64, kl, ku, bs);
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r][u] = fma_c(acc[r][u], rv, g[tr + r * ldg]);
        }
    }
    for (int u = 0; c < nr; c += 64, ++u) {
        const cplx rv = row[c];
        const int64_t tr = tip_row(c, kl, ku, bs);
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r][u] = fma_c(acc[r][u], rv, g[tr + r * ldg]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        cplx t = (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]);
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            t.re += __shfl_xor(t.re, m, 64);
            t.im += __shfl_xor(t.im, m, 64);
        }
        if (lane == 0) z[i + r * ldz] = t;
    }
}

// y_i = g_i - sum_k V[i,k] t_j[k] - sum_k W[i,k] b_{j-1}[k], j the block of row i: one
// thread per row, the tips of the (at most two) blocks of the workgroup's rows staged in
// LDS, four accumulators per row; NR right-hand sides (z + r ldz, g + r ldg,
// y + r ldy) share the loads of V and W.
template <int NR>
__global__ __launch_bounds__(256) void k_part_correct(int64_t n, int64_t n16, int kl, int ku, int64_t bs,
                                                      int64_t nbk, const cplx* __restrict__ V,
                                                      const cplx* __restrict__ W, const cplx* __restrict__ z,
                                                      int64_t ldz, const cplx* __restrict__ g, int64_t ldg,
                                                      cplx* __restrict__ y, int64_t ldy, const int* active) {
    if (active && *active == 0) return;
    extern __shared__ double2 zsm[];
    cplx* zs = reinterpret_cast<cplx*>(zsm);   // NR x 2 x (ku + kl): t_j then b_{j-1}, for blocks jb, jb + 1
    const int w = kl + ku;
    const int64_t r0 = (int64_t)blockIdx.x * 256;
    const int64_t jb = r0 / bs;
    for (int e = threadIdx.x; e < 2 * w; e += 256) {
        const int64_t j = jb + e / w;
        const int q = e % w;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cplx v = mk(0.0, 0.0);
            if (q < ku) {
                if (j <= nbk - 2) v = z[j * w + kl + q + r * ldz];
            } else {
                if (j >= 1 && j <= nbk - 1) v = z[(j - 1) * w + (q - ku) + r * ldz];
            }
            zs[r * 2 * w + e] = v;
        }
    }
    __syncthreads();
    const int64_t i = r0 + threadIdx.x;
    if (i >= n) return;
    const int64_t j = i / bs;
    const int off = (int)(j - jb) * w;          // t_j (ku values), then b_{j-1} (kl values)
    cplx acc[NR][4];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[r][u] = mk(0.0, 0.0);
    if (j <= nbk - 2) {
        int k = 0;
        for (; k + 3 < ku; k += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const cplx v = V[i + (int64_t)(k + u) * n16];
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r][u] = fma_c(acc[r][u], v, zs[r * 2 * w + off + k + u]);
            }
        }
        for (int u = 0; k < ku; ++k, ++u) {
            const cplx v = V[i + (int64_t)k * n16];
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r][u] = fma_c(acc[r][u], v, zs[r * 2 * w + off + k]);
        }
    }
    if (j >= 1) {
        int k = 0;
        for (; k + 3 < kl; k += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const cplx v = W[i + (int64_t)(k + u) * n16];
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r][u] = fma_c(acc[r][u], v, zs[r * 2 * w + off + ku + k + u]);
            }
        }
        for (int u = 0; k < kl; ++k, ++u) {
            const cplx v = W[i + (int64_t)k * n16];
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r][u] = fma_c(acc[r][u], v, zs[r * 2 * w + off + ku + k]);
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
        y[i + r * ldy] = g[i + r * ldg] - ((acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]));
}

constexpr int kSpikeStreams = 4;

// The spike solves' streams: a pool of kPoolStreams per device, made on first use and
// kept for the life of the process.  Each call takes the next kSpikeStreams of them in
// turn, so that calls from several host threads (runs of a batch, factors built ahead)
// mostly get streams of their own; each call orders its own work with events.
constexpr int kPoolStreams = 16;
}  // namespace

simm_status spike_streams(hipStream_t* out) {
    static std::mutex mu;
    static std::map<int, std::array<hipStream_t, kPoolStreams>> pool;
    static unsigned next = 0;
    int dev = 0;
    SIMM_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = pool.find(dev);
    if (it == pool.end()) {
        std::array<hipStream_t, kPoolStreams> a{};
        for (auto& x : a) SIMM_HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        it = pool.emplace(dev, a).first;
    }
    const unsigned first = (next++ % (kPoolStreams / kSpikeStreams)) * kSpikeStreams;
    for (int i = 0; i < kSpikeStreams; ++i) out[i] = it->second[first + i];
    return SIMM_OK;
}

namespace {

simm_status spikes(const SpikeFactor& f, hipStream_t st) {
    const int kl = f.pkl, ku = f.pku, w = kl + ku;
    const int64_t n16 = f.n16;
    const unsigned blocks16 = (unsigned)((n16 + 255) / 256);
    // as many streams as hardware queues (GPU_MAX_HW_QUEUES, 4 unless set), 2 to 4:
    // streams beyond the queues share one and their launches serialise
    int queues = 4;
    if (const char* e = getenv("GPU_MAX_HW_QUEUES")) queues = std::max(1, atoi(e));
    // at most as many streams as fit the device's budget of spinning chain workgroups,
    // held (below, before the streams' release) until they are done
    const int cw = spike_chain_weight(f);
    const int ns = std::max(1, std::min({kSpikeStreams, w, std::max(2, queues), spike_chain_budget() / cw}));
    ChainSlots slots;
    SIMM_TRY(slots.acquire(ns * cw, st));
    hipStream_t ss[kSpikeStreams] = {};
    SIMM_TRY(spike_streams(ss));
    hipEvent_t ev[kSpikeStreams + 1] = {};
    SpikeFactor cl[kSpikeStreams];
    bool have[kSpikeStreams] = {};
    // the clones' scratch comes from st's stream-ordered pool (a plain free would wait for
    // the whole device); it is freed on st once the spike streams are done with it
    struct Release {
        hipStream_t* s;
        hipEvent_t* e;
        SpikeFactor* c;
        bool* h;
        int ns;
        hipStream_t st;
        ~Release() {
            for (int i = 0; i < ns; ++i)
                if (h[i]) (void)hipStreamSynchronize(s[i]);
            for (int i = 0; i < ns; ++i)
                if (h[i]) spike_release_ordered(c[i], st);
            for (int i = 0; i <= ns; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } rel{ss, ev, cl, have, ns, st};
    for (int i = 0; i <= ns; ++i) SIMM_HIP_TRY(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    // up to four coupling columns of one kind per solve, sharing every pass over D's factor
    const int nrmax = spike_max_nrhs(f);
    for (int i = 0; i < ns; ++i) {
        SIMM_TRY(spike_clone_scratch(f, cl[i], st, true, nrmax));
        have[i] = true;
    }
    SIMM_HIP_TRY(hipEventRecord(ev[ns], st));   // D's sweep data and the clones are on st
    for (int i = 0; i < ns; ++i) SIMM_HIP_TRY(hipStreamWaitEvent(ss[i], ev[ns], 0));
    int solve = 0;
    for (int which = 0; which < 2; ++which) {
        const int cols = which == 0 ? ku : kl;
        for (int k0 = 0; k0 < cols;) {
            int nr = nrmax;
            while (nr > cols - k0) nr /= 2;
            const int i = solve++ % ns;
            for (int r = 0; r < nr; ++r)
                hipLaunchKernelGGL(k_part_rhs, dim3(blocks16), dim3(256), 0, ss[i], f.n, n16, kl, ku, f.bs, f.nbk, f.cpl,
                                   which, k0 + r, cl[i].pg + (int64_t)r * n16);
            cplx* out = (which == 0 ? f.Vs : f.Ws) + (int64_t)k0 * n16;
            SIMM_TRY(spike_apply_diag_nr(cl[i], cl[i].pg, n16, out, n16, nr, ss[i]));
            k0 += nr;
        }
    }
    int err = 0;
    for (int i = 0; i < ns; ++i) {
        int e = 0;
        SIMM_HIP_TRY(hipMemcpyAsync(&e, cl[i].err, sizeof(int), hipMemcpyDeviceToHost, ss[i]));
        SIMM_HIP_TRY(hipStreamSynchronize(ss[i]));
        err |= e;
    }
    if (err) {
        set_error("partitioned factorization: a chunk-chain barrier of a spike solve timed out");
        return SIMM_EHIP;
    }
    return SIMM_OK;
}

template <typename CT>
simm_status cut_t(int64_t n, int kl, int ku, CT* AB, int64_t bs, cplx* cpl, hipStream_t st) {
    const int64_t nbk = (n + bs - 1) / bs;
    if (nbk < 2) return SIMM_OK;
    hipLaunchKernelGGL(k_part_cut<CT>, dim3((unsigned)(nbk - 1)), dim3(256), 0, st, n, kl, ku, AB, bs, cpl);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace

simm_status part_cut(int64_t n, int kl, int ku, cplx* AB, int64_t bs, cplx* cpl, hipStream_t st) {
    return cut_t(n, kl, ku, AB, bs, cpl, st);
}
simm_status part_cut(int64_t n, int kl, int ku, cplxf* AB, int64_t bs, cplx* cpl, hipStream_t st) {
    return cut_t(n, kl, ku, AB, bs, cpl, st);
}

simm_status part_prepare(SpikeFactor& f, hipStream_t st) {
    const int kl = f.kl, ku = f.ku, w = kl + ku;
    f.pkl = kl;
    f.pku = ku;
    f.nbk = (f.n + f.bs - 1) / f.bs;
    f.nr = (f.nbk - 1) * (int64_t)w;
    const int64_t n16 = f.n16, nr = f.nr;
    const int klr = 2 * kl + ku - 1, kur = kl + 2 * ku - 1;
    if (f.nbk < 2 || nr > kPartMaxReduced || lu_panel_width(klr) == 0) {
        set_error("partitioned factorization: block layout out of range");
        return SIMM_EUNSUPPORTED;
    }
    const size_t elems = (size_t)n16 * w + (size_t)nr * nr + (size_t)n16 + (size_t)nr + 64;
    SIMM_HIP_TRY(device_malloc(&f.part_mem, sizeof(cplx) * elems + 8 * 256));
    char* p = reinterpret_cast<char*>(f.part_mem);
    auto take = [&](size_t count) {
        char* r = p;
        p += (sizeof(cplx) * count + 255) & ~(size_t)255;
        return reinterpret_cast<cplx*>(r);
    };
    f.Vs = take((size_t)n16 * ku);
    f.Ws = take((size_t)n16 * kl);
    f.Rinv = take((size_t)nr * nr);
    f.pg = take((size_t)n16);
    f.pz = take((size_t)nr);
    // SIMM_PART_TIMING: the phases' times on stderr
    const bool timing = getenv("SIMM_PART_TIMING") != nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    auto stamp = [&](const char* what, std::chrono::steady_clock::time_point& since) {
        if (!timing) return;
        (void)hipStreamSynchronize(st);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[simm part] n = %lld, %lld blocks of %lld: %s %.2f ms\n", (long long)f.n,
                     (long long)f.nbk, (long long)f.bs, what,
                     std::chrono::duration<double, std::milli>(now - since).count());
        since = now;
    };
    auto tp = t0;
    // spikes: one solve with D's factor per coupling column, the columns dealt to
    // kSpikeStreams streams (each with its own sweep scratch and right-hand side), since
    // one solve is a chain of latency-bound launches that fills little of the device
    SIMM_TRY(spikes(f, st));
    stamp("spikes", tp);
    // the reduced system, its band LU and its inverse
    const int ldr = 2 * klr + kur + 1;
    cplx *ABr = nullptr, *LPr = nullptr;
    int *ipr = nullptr, *info = nullptr;
    // temporaries in st's order (freed there, no device-wide wait)
    struct Free {
        void* q[4];
        hipStream_t st;
        ~Free() {
            for (void* x : q)
                if (x) (void)hipFreeAsync(x, st);
        }
    } fr{{nullptr, nullptr, nullptr, nullptr}, st};
    SIMM_HIP_TRY(device_malloc_async((void**)&ABr, sizeof(cplx) * ((size_t)ldr * nr + 1), st));
    fr.q[0] = ABr;
    SIMM_HIP_TRY(device_malloc_async((void**)&LPr, sizeof(cplx) * band_lu_panel_elems(nr, klr), st));
    fr.q[1] = LPr;
    SIMM_HIP_TRY(device_malloc_async((void**)&ipr, sizeof(int) * (size_t)((nr + 15) / 16 * 16), st));
    fr.q[2] = ipr;
    SIMM_HIP_TRY(device_malloc_async((void**)&info, sizeof(int), st));
    fr.q[3] = info;
    SIMM_HIP_TRY(hipMemsetAsync(ABr, 0, sizeof(cplx) * ((size_t)ldr * nr + 1), st));
    const int info0 = INT_MAX;
    SIMM_HIP_TRY(hipMemcpyAsync(info, &info0, sizeof(int), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_part_reduced, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, nr, kl, ku, f.bs, f.nbk,
                       n16, (const cplx*)f.Vs, (const cplx*)f.Ws, ABr, klr, kur);
    SIMM_HIP_TRY(hipGetLastError());
    SIMM_TRY(band_lu(nr, klr, kur, ABr, ipr, LPr, info, st));
    stamp("reduced system and its LU", tp);
    int info_h = 0;
    SIMM_HIP_TRY(hipMemcpyAsync(&info_h, info, sizeof(int), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    if (info_h != INT_MAX) {
        set_error("partitioned factorization: the reduced system is singular");
        return SIMM_ESINGULAR_SHIFT;
    }
    hipLaunchKernelGGL(k_part_inverse, dim3((unsigned)nr), dim3(256), sizeof(cplx) * (size_t)nr, st, nr, klr, kur,
                       (const cplx*)ABr, (const int*)ipr, f.Rinv);
    SIMM_HIP_TRY(hipGetLastError());
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    stamp("reduced inverse", tp);
    return SIMM_OK;
}

namespace {
template <int NR>
void part_tail(const SpikeFactor& f, cplx* y, int64_t ldy, const int* active, hipStream_t st) {
    hipLaunchKernelGGL((k_part_tips<NR>), dim3((unsigned)((f.nr + 3) / 4)), dim3(256), 0, st, f.nr, f.pkl, f.pku, f.bs,
                       (const cplx*)f.Rinv, (const cplx*)f.pg, f.n16, f.pz, f.nr, active);
    hipLaunchKernelGGL((k_part_correct<NR>), dim3((unsigned)((f.n + 255) / 256)), dim3(256),
                       sizeof(cplx) * 2 * (size_t)(f.pkl + f.pku) * NR, st, f.n, f.n16, f.pkl, f.pku, f.bs, f.nbk,
                       (const cplx*)f.Vs, (const cplx*)f.Ws, (const cplx*)f.pz, f.nr, (const cplx*)f.pg, f.n16, y, ldy,
                       active);
}
}  // namespace

simm_status part_apply(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st) {
    SIMM_TRY(spike_apply_diag(f, u, f.pg, active, st));
    part_tail<1>(f, y, f.n16, active, st);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status part_apply_nr(const SpikeFactor& f, const cplx* u, int64_t ldu, cplx* y, int64_t ldy, int nr,
                          hipStream_t st) {
    // g = D^{-1} u for the nr columns (f.pg and f.pz hold f.nrhs columns each)
    SIMM_TRY(spike_apply_diag_nr(f, u, ldu, f.pg, f.n16, nr, st));
    if (nr == 4) part_tail<4>(f, y, ldy, nullptr, st);
    else if (nr == 2) part_tail<2>(f, y, ldy, nullptr, st);
    else part_tail<1>(f, y, ldy, nullptr, st);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
