// Partitioned, blocked application of the band LU factor: y = U^{-1} L^{-1} P u
// (the Cayley operator of Sec. 2, eq. (IMxb), is M x = U^{-1} L^{-1} P B x).
//
// A sweep over the columns is a linear state machine: before column J of the
// forward sweep the rows still receiving updates are J .. J+kl-1 (kl values, the
// "state"), and before column J-1 of the backward sweep they are J-K .. J-1
// (K = effective upper bandwidth of U).  The columns are cut into P chunks of s
// columns.  For chunk c, with state t_c at its start and its input rows,
//     [y_c ; t_{c+1}] = [y0_c ; tau_c] + [Psi_c ; Phi_c] t_c,
// where (y0_c, tau_c) is the chunk's response to its input with a zero state and
// Psi_c, Phi_c its response to a unit state.  Per application:
//   1. all chunks in parallel: zero-state chunk sweeps -> y0_c, tau_c;
//   2. the chain t_{c+1} = tau_c + Phi_c t_c (P steps of a K x K product),
//      run by a few workgroups that meet at a device-scope barrier per step;
//   3. all rows in parallel: y_c = y0_c + Psi_c t_c.
// Psi_c and Phi_c depend only on the factor and are formed once per shift by the
// same chunk kernels run with unit states.  This is the partitioning idea of
// Polizzi and Sameh's SPIKE algorithm, applied to the triangular factors (the
// factorization itself is the ordinary band LU with partial pivoting).
//
// Inside a chunk the sweep advances 16 columns (one LU panel) at a time.  For the
// forward sweep the window is the 16 + kl rows the panel touches: its 16
// interchanges permute the window, the top 16 rows become y = L11^{-1} top and the
// rest receive -L21 L11^{-1} top.  With the per-panel blocks Gf = [L11^{-1};
// -L21 L11^{-1}] formed once per shift, every window row is one 16-term product
// with the 16 top values: no sequential triangular solve in the loop.  The
// backward sweep does the same with Hb = [-U12 U11^{-1}; U11^{-1}] on the K + 16
// rows above and in the panel.  One thread per window row keeps its value in a
// register; per panel the rows meet once in LDS (one barrier), and the 16 values
// every row needs are read by 16 lanes and broadcast with lane reads.  The matrix
// is extended by identity to n16 = 16 ceil(n / 16) rows.
#include <array>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

__device__ inline cplx ldz(const cplx* p, int64_t i, int64_t n) { return (i >= 0 && i < n) ? p[i] : mk(0.0, 0.0); }

__device__ inline cplx ldsr(const cplx* p) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    return cplx{v.x, v.y};
}
__device__ inline void ldsw(cplx* p, cplx v) { *reinterpret_cast<double2*>(p) = double2{v.re, v.im}; }

__device__ inline double rdl(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ inline cplx rdl(cplx v, int l) { return cplx{rdl(v.re, l), rdl(v.im, l)}; }

// Window position that row i held before the interchanges (t, pv[t]), t = 0..15,
// were applied in order.
__device__ inline int trace_src16(int i, const int* pv) {
    int pos = i;
#pragma unroll
    for (int t = 15; t >= 0; --t) {
        const int p = pv[t];
        pos = (pos == t) ? p : ((pos == p) ? t : pos);
    }
    return pos;
}

}  // namespace

// ---------------------------------------------------------------------------
// per-panel blocks (once per shift)
// ---------------------------------------------------------------------------
// Gf[p] = [L11^{-1}; -L21 L11^{-1}] from the LU's permuted multipliers of panel p.
template <typename LT, typename GT>
__global__ __launch_bounds__(512) void k_blocks_fwd(int kl, const LT* __restrict__ LP, GT* __restrict__ Gf) {
    __shared__ cplx L11[16 * 17], Li[16 * 17];
    const int RW = kl + 16;
    const int64_t p = blockIdx.x;
    const int r = threadIdx.x;
    cplx lr[16];
    if (r < RW) {
#pragma unroll
        for (int q = 0; q < 16; ++q) lr[q] = widen(LP[(p * 16 + q) * RW + r]);
        if (r < 16) {
#pragma unroll
            for (int q = 0; q < 16; ++q) L11[r * 17 + q] = lr[q];
        }
    }
    __syncthreads();
    if (r < 16) {   // column r of L11^{-1} (unit lower triangular)
        cplx x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            cplx acc = mk(i == r ? 1.0 : 0.0, 0.0);
#pragma unroll
            for (int k = 0; k < i; ++k) acc = fms(acc, L11[i * 17 + k], x[k]);
            x[i] = (i < r) ? mk(0.0, 0.0) : acc;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Li[i * 17 + r] = x[i];
    }
    __syncthreads();
    if (r < RW) {
        cplx g[16];
        if (r < 16) {
#pragma unroll
            for (int q = 0; q < 16; ++q) g[q] = Li[r * 17 + q];
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                cplx acc = mk(0.0, 0.0);
#pragma unroll
                for (int k = 0; k < 16; ++k) acc = fms(acc, lr[k], Li[k * 17 + q]);
                g[q] = acc;
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) Gf[(p * 16 + q) * RW + r] = narrow<GT>(g[q]);
    }
}

// Hb[p] = [-U(j0-K .. j0-1, j0 .. j0+15) U11^{-1}; U11^{-1}], U11 = U(j0 .., j0 ..),
// the identity past row n.
template <typename AT, typename GT>
__global__ __launch_bounds__(1024) void k_blocks_bwd(int64_t n, int K, int kv, int ldab, const AT* __restrict__ AB,
                                                     GT* __restrict__ Hb) {
    __shared__ cplx U11[16 * 17], Ui[16 * 17];
    const int RW = K + 16;
    const int64_t p = blockIdx.x;
    const int64_t j0 = 16 * p;
    const int r = threadIdx.x;
    auto U = [&](int64_t i, int64_t j) -> cplx {   // U(i, j) for j >= i (zero outside the stored band)
        if (j >= n || i >= n) return mk(i == j ? 1.0 : 0.0, 0.0);
        if (i < 0 || j - i > kv) return mk(0.0, 0.0);
        return widen(AB[(int64_t)(kv + i - j) + j * ldab]);
    };
    if (r < 256) {
        const int i = r >> 4, q = r & 15;
        U11[i * 17 + q] = (q >= i) ? U(j0 + i, j0 + q) : mk(0.0, 0.0);
    }
    __syncthreads();
    if (r < 16) {   // column r of U11^{-1} by back substitution
        cplx x[16];
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            cplx acc = mk(i == r ? 1.0 : 0.0, 0.0);
#pragma unroll
            for (int k = i + 1; k < 16; ++k) acc = fms(acc, U11[i * 17 + k], x[k]);
            x[i] = (i > r) ? mk(0.0, 0.0) : cdiv(acc, U11[i * 17 + i]);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Ui[i * 17 + r] = x[i];
    }
    __syncthreads();
    if (r < RW) {
        cplx h[16];
        if (r >= K) {
#pragma unroll
            for (int q = 0; q < 16; ++q) h[q] = Ui[(r - K) * 17 + q];
        } else {
            const int64_t row = j0 - K + r;
            cplx ur[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) ur[k] = U(row, j0 + k);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                cplx acc = mk(0.0, 0.0);
#pragma unroll
                for (int k = 0; k < 16; ++k) acc = fms(acc, ur[k], Ui[k * 17 + q]);
                h[q] = acc;
            }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) Hb[(p * 16 + q) * RW + r] = narrow<GT>(h[q]);
    }
}

// ---------------------------------------------------------------------------
// forward (L) chunk sweep, 16 columns per step
// ---------------------------------------------------------------------------
// NR right-hand sides per workgroup share every panel block it loads: NR unit vectors
// r0 .. r0+NR-1 (r0 = NR blockIdx.y) for the unit-state responses, or NR input columns
// for zero-state sweeps (each column computed as with NR = 1).
// Panels of block rows loaded ahead by the chunk sweeps: two for the single-vector
// FP64 sweeps of up to 512 threads (a third register set of 64 VGPRs fits), else one.
template <int T, int NR, typename GT>
constexpr int prefetch_depth() {
    return (NR == 1 && T <= 512 && std::is_same<GT, cplx>::value) ? 2 : 1;
}

template <int T, int NR, typename GT>
__global__ __launch_bounds__(T) void k_chunk_fwd(SpikeFwdT<GT> a) {
    if (a.active != nullptr && *a.active == 0) return;
    extern __shared__ double2 sraw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int kl = a.kl, RW = kl + 16;
    const int c = blockIdx.x, r0 = blockIdx.y * NR;
    const int64_t J0 = (int64_t)c * a.s, J1 = min(a.n16, J0 + a.s);
    const int len = (int)(J1 - J0);
    const int npan = len / 16;
    // LDS: window values by slot (2 x NR x RW, alternating per panel), the chunk's
    // outputs (NR x len), its input rows J0+kl .. J1+RW-1 (len + 16; NR columns of them
    // in mode 0) and its pivots (len).  Several zero-state columns write their outputs
    // over their inputs: the output of step i (entry 16 i + pos) replaces an input read
    // at an earlier step (or before the first), across a barrier.
    const int NI = (a.mode == 0) ? NR : 1;
    const bool inplace = NR > 1 && a.mode == 0;
    cplx* S = reinterpret_cast<cplx*>(sraw);
    cplx* outb = S + 2 * NR * RW;
    cplx* inb = outb + (inplace ? 0 : NR * len);
    auto outc = [&](int u) { return inplace ? inb + u * (len + 16) : outb + u * len; };
    int* pivb = reinterpret_cast<int*>(inb + NI * (len + 16));
    for (int q = tid; q < len; q += T) pivb[q] = a.ipiv[J0 + q] - (int)(J0 + (q & ~15));
    for (int q = tid; q < len + 16; q += T) {
        const int64_t row = J0 + kl + q;
        for (int u = 0; u < NI; ++u)
            inb[u * (len + 16) + q] = (a.mode == 0 && row < a.n) ? a.u[row + u * a.ldu] : mk(0.0, 0.0);
    }
    __syncthreads();
    const bool mine = tid < RW;
    // thread tid owns LDS slot tid; the row in it has window position pos; the slot
    // of position 0 is `off`
    int pos = tid, off = 0;
    cplx val[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        val[u] = mk(0.0, 0.0);
        if (mine) val[u] = (a.mode == 0) ? ((pos >= kl) ? inb[u * (len + 16) + pos - kl] : mk(0.0, 0.0))
                                         : mk(pos == r0 + u ? 1.0 : 0.0, 0.0);
    }
    const int64_t p0 = J0 / 16;
    // The block row of my position PD panels ahead is loaded PD panels ahead, into one
    // of PD + 1 register sets (a load takes longer than a panel step); no global load
    // sits in a branch, so the waits for what a step consumes never wait for what it
    // prefetches.
    constexpr int PD = prefetch_depth<T, NR, GT>();
    const int64_t plast = a.n16 / 16 - 1;
    auto adv = [&](int ps) { return (ps >= 16) ? ps - 16 : ps + RW - 16; };
    cplx gA[16], gB[16], gC[PD == 2 ? 16 : 1];
    auto prefetch = [&](auto& g, int64_t p, int ps) {
        const GT* gp = a.G + p * 16 * RW + (mine ? ps : 0);
#pragma unroll
        for (int q = 0; q < 16; ++q) g[q] = widen(gp[q * RW]);
    };
    prefetch(gA, p0, pos);
    if constexpr (PD == 2) prefetch(gB, min(p0 + 1, plast), adv(pos));
    auto step = [&](int i, auto& gc, auto& gn) {
        const int64_t p = p0 + i;
        const int buf = i & 1;
        const int pos_n = adv(pos);
        // unconditional: no branch around loads
        if constexpr (PD == 2) prefetch(gn, min(p + 2, plast), adv(pos_n));
        else prefetch(gn, min(p + 1, plast), pos_n);
        if (mine) {
#pragma unroll
            for (int u = 0; u < NR; ++u) ldsw(S + (buf * NR + u) * RW + tid, val[u]);
        }
        lds_barrier();
        int pv[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) pv[t] = pivb[16 * i + t];
        auto slot = [&](int ps) {
            const int sl = ps + off;
            return sl >= RW ? sl - RW : sl;
        };
        const int sv = slot(trace_src16(mine ? pos : 0, pv)), st = slot(trace_src16(lane & 15, pv));
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const cplx v2 = ldsr(S + (buf * NR + u) * RW + sv);
            const cplx tq = ldsr(S + (buf * NR + u) * RW + st);
            cplx acc = (pos >= 16) ? v2 : mk(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 16; ++q) acc = fma_c(acc, gc[q], rdl(tq, q));
            if (mine) {
                if (pos < 16) {
                    ldsw(outc(u) + 16 * i + pos, acc);
                    // row J0 + 16 i + RW + pos enters (zero in mode 1)
                    val[u] = inb[(a.mode == 0 ? u : 0) * (len + 16) + 16 * i + 16 + pos];
                } else {
                    val[u] = acc;
                }
            }
        }
        pos = pos_n;
        off = (off + 16 >= RW) ? off + 16 - RW : off + 16;
    };
    int i = 0;
    if constexpr (PD == 2) {
        for (; i + 3 <= npan; i += 3) {
            step(i, gA, gC);
            step(i + 1, gB, gA);
            step(i + 2, gC, gB);
        }
        if (i < npan) step(i, gA, gC);
        if (i + 1 < npan) step(i + 1, gB, gA);
    } else {
        for (; i + 2 <= npan; i += 2) {
            step(i, gA, gB);
            step(i + 1, gB, gA);
        }
        if (i < npan) step(i, gA, gB);
    }
    // end state: rows J1 .. J1+kl-1 hold positions 0 .. kl-1
    if (mine && pos < kl) {
        if (a.mode == 0) {
#pragma unroll
            for (int u = 0; u < NR; ++u) a.tau[(int64_t)c * kl + pos + u * a.ldt] = val[u];
        } else {
#pragma unroll
            for (int u = 0; u < NR; ++u)   // Phi_c(i, r) at [c][i][r]
                if (r0 + u < kl) a.Phi[((int64_t)c * kl + pos) * kl + r0 + u] = val[u];
        }
    }
    __syncthreads();
    if (a.mode == 0) {
#pragma unroll
        for (int u = 0; u < NR; ++u)
            for (int q = tid; q < len; q += T) {
                const cplx v = ldsr(outc(u) + q);
                if (J0 + q < a.n) a.y[J0 + q + u * a.ldy] = v;
            }
    } else {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            if (r0 + u >= kl) continue;
            for (int q = tid; q < len; q += T)
                a.Psi[J0 + q + (int64_t)(r0 + u) * a.n16] = narrow<GT>(ldsr(outb + u * len + q));
        }
    }
}

// ---------------------------------------------------------------------------
// backward (U) chunk sweep, 16 columns per step (bottom panel first)
// ---------------------------------------------------------------------------
template <int T, int NR, typename GT>
__global__ __launch_bounds__(T) void k_chunk_bwd(SpikeBwdT<GT> a) {
    if (a.active != nullptr && *a.active == 0) return;
    extern __shared__ double2 sraw[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int K = a.K, RW = K + 16;
    const int c = blockIdx.x, r0 = blockIdx.y * NR;
    const int64_t J0 = (int64_t)c * a.s, J1 = min(a.n16, J0 + a.s);
    const int len = (int)(J1 - J0);
    const int npan = len / 16;
    // LDS: window (2 x NR x RW), outputs (NR x len), input rows J0-K-16 .. J1-K-1 (len + 16;
    // NR columns of them in mode 0).  Several zero-state columns write their outputs over
    // their inputs: a step's output entry is the entry its thread reads the entering row
    // from, read first.
    const int NI = (a.mode == 0) ? NR : 1;
    const bool inplace = NR > 1 && a.mode == 0;
    cplx* S = reinterpret_cast<cplx*>(sraw);
    cplx* outb = S + 2 * NR * RW;
    cplx* inb = outb + (inplace ? 0 : NR * len);
    auto outc = [&](int u) { return inplace ? inb + u * (len + 16) : outb + u * len; };
    const int64_t in0 = J0 - K - 16;
    for (int q = tid; q < len + 16; q += T) {
        const int64_t row = in0 + q;
        for (int u = 0; u < NI; ++u)
            inb[u * (len + 16) + q] = (a.mode == 0 && row >= 0 && row < a.n) ? a.z[row + u * a.ldu] : mk(0.0, 0.0);
    }
    __syncthreads();
    const bool mine = tid < RW;
    // window of the panel at j0: rows j0-K .. j0+15 at positions 0 .. K+15; the
    // state rows of the chunk end (J1-K .. J1-1) start at positions 16 .. K+15
    int pos = tid, off = 0;
    const int64_t pl = J1 / 16 - 1;             // first (lowest) panel
    cplx val[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        val[u] = mk(0.0, 0.0);
        if (mine) val[u] = (a.mode == 0) ? ((pos < 16) ? inb[u * (len + 16) + (16 * pl - K + pos) - in0] : mk(0.0, 0.0))
                                         : mk(pos - 16 == r0 + u ? 1.0 : 0.0, 0.0);
    }
    // prefetch PD panels ahead, as in the forward sweep
    constexpr int PD = prefetch_depth<T, NR, GT>();
    auto adv = [&](int ps) { return (ps < K) ? ps + 16 : ps - K; };
    cplx hA[16], hB[16], hC[PD == 2 ? 16 : 1];
    auto prefetch = [&](auto& h, int64_t p, int ps) {
        const GT* hp = a.H + p * 16 * RW + (mine ? ps : 0);
#pragma unroll
        for (int q = 0; q < 16; ++q) h[q] = widen(hp[q * RW]);
    };
    prefetch(hA, pl, pos);
    if constexpr (PD == 2) prefetch(hB, max(pl - 1, (int64_t)0), adv(pos));
    auto step = [&](int i, auto& hc, auto& hn) {
        const int64_t p = pl - i;
        const int buf = i & 1;
        const int pos_n = adv(pos);
        // unconditional: no branch around loads
        if constexpr (PD == 2) prefetch(hn, max(p - 2, (int64_t)0), adv(pos_n));
        else prefetch(hn, max(p - 1, (int64_t)0), pos_n);
        if (mine) {
#pragma unroll
            for (int u = 0; u < NR; ++u) ldsw(S + (buf * NR + u) * RW + tid, val[u]);
        }
        lds_barrier();
        int sl = K + (lane & 15) + off;
        sl = sl >= RW ? sl - RW : sl;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const cplx bq = ldsr(S + (buf * NR + u) * RW + sl);
            cplx acc = (pos < K) ? val[u] : mk(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 16; ++q) acc = fma_c(acc, hc[q], rdl(bq, q));
            if (mine) {
                if (pos >= K) {
                    // row j0-16-K + (pos-K) enters (zero in mode 1)
                    const cplx enter = inb[(a.mode == 0 ? u : 0) * (len + 16) + (16 * p - 16 - K + pos - K) - in0];
                    ldsw(outc(u) + (16 * p - J0) + pos - K, acc);
                    val[u] = enter;
                } else {
                    val[u] = acc;
                }
            }
        }
        pos = pos_n;
        off = (off >= 16) ? off - 16 : off + RW - 16;
    };
    int i = 0;
    if constexpr (PD == 2) {
        for (; i + 3 <= npan; i += 3) {
            step(i, hA, hC);
            step(i + 1, hB, hA);
            step(i + 2, hC, hB);
        }
        if (i < npan) step(i, hA, hC);
        if (i + 1 < npan) step(i + 1, hB, hA);
    } else {
        for (; i + 2 <= npan; i += 2) {
            step(i, hA, hB);
            step(i + 1, hB, hA);
        }
        if (i < npan) step(i, hA, hB);
    }
    // end state: rows J0-K .. J0-1 hold positions 16 .. K+15
    if (mine && pos >= 16) {
        if (a.mode == 0) {
#pragma unroll
            for (int u = 0; u < NR; ++u) a.tau[(int64_t)c * K + pos - 16 + u * a.ldt] = val[u];
        } else {
#pragma unroll
            for (int u = 0; u < NR; ++u)
                if (r0 + u < K) a.Phi[((int64_t)c * K + pos - 16) * K + r0 + u] = val[u];
        }
    }
    __syncthreads();
    if (a.mode == 0) {
#pragma unroll
        for (int u = 0; u < NR; ++u)
            for (int q = tid; q < len; q += T) {
                const cplx v = ldsr(outc(u) + q);
                if (J0 + q < a.n) a.y[J0 + q + u * a.ldy] = v;
            }
    } else {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            if (r0 + u >= K) continue;
            for (int q = tid; q < len; q += T)
                a.Psi[J0 + q + (int64_t)(r0 + u) * a.n16] = narrow<GT>(ldsr(outb + u * len + q));
        }
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
constexpr int SPIKE_CTR_STRIDE = 64;   // unsigned counters 256 bytes apart

// CH_PARTS threads per state row, CH_THREADS / CH_PARTS rows per workgroup.
// Groups (blockIdx.y) run independent chains over their L chunks (chain order q:
// chunk q forward, P-1-q backward): group 0 from the true initial state, the others
// from zero; each group meets at its own barrier counter and leaves the state after
// its last chunk in gout (the last group stops one step earlier: no chunk follows).
template <int MAXQ, int CH_PARTS, int NR>
__global__ __launch_bounds__(CH_THREADS) void k_spike_chain(SpikeChain a) {
    constexpr int CH_ROWS = CH_THREADS / CH_PARTS;
    static_assert(CH_ROWS <= 64, "wave 0 stores the workgroup's rows");
    if (a.active != nullptr && *a.active == 0) return;
    __shared__ cplx tcur[NR][CH_PARTS * MAXQ];       // states (NR right-hand sides), zero-padded
    __shared__ cplx rows_out[NR][CH_ROWS];           // this workgroup's rows of the next states
    const int K = a.K;
    const int g = blockIdx.x;
    const int64_t grp = blockIdx.y;
    const int tid = threadIdx.x;
    const int il = tid / CH_PARTS, part = tid % CH_PARTS;
    const int i = g * CH_ROWS + il;
    const int ic = min(i, K - 1);
    const int64_t KK = (int64_t)K * K;
    const int64_t q0 = grp * a.L, q1 = min(a.P, q0 + a.L);
    const int64_t nsteps = (q1 == a.P) ? q1 - q0 - 1 : q1 - q0;
    auto chunk = [&](int64_t q) { return a.forward ? q : a.P - 1 - q; };
    unsigned* counter = a.counter + grp * SPIKE_CTR_STRIDE;
    for (int r = tid; r < CH_PARTS * MAXQ; r += CH_THREADS) {
        const int64_t row = a.init_row0 + r;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const cplx v = (r < K && grp == 0) ? ldz(a.init_src + u * a.ldi, row, a.n) : mk(0.0, 0.0);
            tcur[u][r] = v;
            if (g == 0 && r < K) a.t[chunk(q0) * K + r + u * a.ldt] = v;
        }
    }
    // Several right-hand sides with the longer states read their Phi row in halves of 16
    // per step, not ahead (the whole row ahead beside the states' accumulators would spill
    // registers); the accumulation order is the same.
    constexpr bool SPLIT = NR > 1 && MAXQ > 16;
    cplx ph[SPLIT ? 16 : MAXQ];
    auto load_phi = [&](int64_t c) {
        const cplx* prow = a.Phi + c * KK + (int64_t)ic * K;
#pragma unroll
        for (int q = 0; q < (SPLIT ? 16 : MAXQ); ++q) ph[q] = prow[min(part + CH_PARTS * q, K - 1)];
    };
    if (!SPLIT && nsteps > 0) load_phi(chunk(q0));
    __syncthreads();
    for (int64_t step = 0; step < nsteps; ++step) {
        const int64_t q = q0 + step;
        const int64_t c = chunk(q);
        // destination of the next states: the next chunk of the group, or the group output
        const bool to_t = q + 1 < q1;
        cplx* dst = to_t ? a.t + chunk(q + 1) * K : a.gout + grp * K;
        const int64_t ldd = to_t ? a.ldt : a.ldg;
        cplx acc[NR];
#pragma unroll
        for (int u = 0; u < NR; ++u) acc[u] = mk(0.0, 0.0);
        if constexpr (SPLIT) {
            const cplx* prow = a.Phi + c * KK + (int64_t)ic * K;
#pragma unroll
            for (int h = 0; h < MAXQ / 16; ++h) {
#pragma unroll
                for (int q = 0; q < 16; ++q) ph[q] = prow[min(part + CH_PARTS * (16 * h + q), K - 1)];
#pragma unroll
                for (int q = 0; q < 16; ++q)
#pragma unroll
                    for (int u = 0; u < NR; ++u)
                        acc[u] = fma_c(acc[u], ph[q], tcur[u][part + CH_PARTS * (16 * h + q)]);   // padded t is 0
            }
        } else {
#pragma unroll
            for (int qq = 0; qq < MAXQ; ++qq)
#pragma unroll
                for (int u = 0; u < NR; ++u)
                    acc[u] = fma_c(acc[u], ph[qq], tcur[u][part + CH_PARTS * qq]);   // padded t is 0
            if (step + 1 < nsteps) load_phi(chunk(q + 1));
        }
#pragma unroll
        for (int u = 0; u < NR; ++u) {
#pragma unroll
            for (int m = CH_PARTS / 2; m >= 1; m >>= 1) {
                acc[u].re += __shfl_xor(acc[u].re, m, 64);
                acc[u].im += __shfl_xor(acc[u].im, m, 64);
            }
            if (part == 0 && i < K) rows_out[u][il] = a.tau[c * K + i + u * a.ldt] + acc[u];
        }
        __syncthreads();
        // Device-scope barrier of the group.  Wave 0 alone exchanges the states with the
        // other workgroups: it stores this workgroup's rows, releases them (one agent-scope
        // release), arrives, polls with relaxed loads (an acquiring load would invalidate
        // the XCD's L2 on every poll), acquires once and loads the whole next states into
        // LDS.  The other waves meet it at the workgroup barriers.  One write-back and one
        // invalidate per workgroup and step: they serialise per XCD, so fences from every
        // wave slowed concurrent chains several-fold.
        if (tid < 64) {
            if (tid < CH_ROWS && g * CH_ROWS + tid < K) {
#pragma unroll
                for (int u = 0; u < NR; ++u) dst[g * CH_ROWS + tid + u * ldd] = rows_out[u][tid];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (tid == 0) {
                __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned target = (unsigned)(gridDim.x * (step + 1));
                long spins = 0;
                while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > 40000000L) {
                        atomicExch(a.err, 1);
                        break;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            // all loads in flight at once (indices clamped into the state), then to LDS
            constexpr int NL = (CH_PARTS * MAXQ + 63) / 64;
            if constexpr (NR == 1 || MAXQ <= 16) {
                cplx nxt[NR][NL];
#pragma unroll
                for (int u = 0; u < NR; ++u)
#pragma unroll
                    for (int v = 0; v < NL; ++v) nxt[u][v] = dst[min(tid + 64 * v, K - 1) + u * ldd];
#pragma unroll
                for (int u = 0; u < NR; ++u)
#pragma unroll
                    for (int v = 0; v < NL; ++v)
                        tcur[u][tid + 64 * v] = csel(tid + 64 * v < K, nxt[u][v], mk(0.0, 0.0));   // padding stays 0
            } else {
                // the longer states of several right-hand sides one after another (all of
                // them in flight at once would spill the registers that hold phi)
#pragma unroll
                for (int u = 0; u < NR; ++u) {
                    cplx nxt[NL];
#pragma unroll
                    for (int v = 0; v < NL; ++v) nxt[v] = dst[min(tid + 64 * v, K - 1) + u * ldd];
#pragma unroll
                    for (int v = 0; v < NL; ++v) tcur[u][tid + 64 * v] = csel(tid + 64 * v < K, nxt[v], mk(0.0, 0.0));
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        __syncthreads();
    }
    // Leave the group's counters at zero for the next launch on this factor: every
    // workgroup has left its last poll when it arrives here, so the last to arrive
    // (second counter of the group's line) clears both.
    if (nsteps > 0 && tid == 0) {
        unsigned* leave = counter + 1;
        const unsigned prev = __hip_atomic_fetch_add(leave, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(leave, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Second level of the chain: the true start state T_g of every group g >= 1 (from the
// chain over groups) enters its chunks through the transfer products,
//     t_q += Pi_q T_g   (Pi_q = Phi_{q-1} ... Phi_{q0(g)}, chain order; Pi_{q0} = I),
// 16 threads per state row, 16 rows per workgroup, blockIdx.y = chain-order chunk q.
template <int MAXQ, int NR>
__global__ __launch_bounds__(256) void k_spike_fix(int K, int64_t P, int64_t L, int forward, const cplx* __restrict__ Pi,
                                                   const cplx* __restrict__ tg, cplx* __restrict__ t, int64_t ldg,
                                                   int64_t ldt, const int* active) {
    if (active != nullptr && *active == 0) return;
    const int64_t q = blockIdx.y;
    const int64_t grp = q / L;
    if (grp == 0) return;
    __shared__ cplx Ts[NR][16 * MAXQ];
    const int tid = threadIdx.x, il = tid >> 4, part = tid & 15;
    const int i = blockIdx.x * 16 + il;
    for (int r = tid; r < 16 * MAXQ; r += 256) {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const cplx* T = tg + (grp - 1) * K + u * ldg;    // true state at the group's first chunk
            Ts[u][r] = (r < K) ? T[r] : mk(0.0, 0.0);
        }
    }
    __syncthreads();
    const int64_t c = forward ? q : P - 1 - q;
    if (q == grp * L) {
        // first chunk of the group: its chain ran from zero, so its state is T_g itself
        if (part == 0 && i < K) {
#pragma unroll
            for (int u = 0; u < NR; ++u) t[c * K + i + u * ldt] = Ts[u][i];
        }
        return;
    }
    const cplx* prow = Pi + q * (int64_t)K * K + (int64_t)min(i, K - 1) * K;
    cplx acc[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) acc[u] = mk(0.0, 0.0);
#pragma unroll
    for (int qq = 0; qq < MAXQ; ++qq) {
        const int r = part + 16 * qq;
        const cplx pv = prow[min(r, K - 1)];
#pragma unroll
        for (int u = 0; u < NR; ++u) acc[u] = fma_c(acc[u], pv, Ts[u][r]);          // padded T is 0
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) {
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) {
            acc[u].re += __shfl_xor(acc[u].re, m, 64);
            acc[u].im += __shfl_xor(acc[u].im, m, 64);
        }
        if (part == 0 && i < K) t[c * K + i + u * ldt] = t[c * K + i + u * ldt] + acc[u];
    }
}

// Copies of the group's first transfer matrix: Pi_{q0+1} = Phi_{chunk(q0)}, groups 1..ng.
__global__ __launch_bounds__(256) void k_pi_first(int K, int64_t P, int64_t L, int forward, int64_t ng,
                                                  const cplx* __restrict__ Phi, cplx* __restrict__ Pi) {
    const int64_t KK = (int64_t)K * K;
    const int64_t grp = 1 + blockIdx.y;
    if (grp > ng) return;
    const int64_t q = grp * L;
    const int64_t c = forward ? q : P - 1 - q;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < KK; e += (int64_t)gridDim.x * 256)
        Pi[(q + 1) * KK + e] = Phi[c * KK + e];
}

// y(j) += sum_r Psi(j, r) t_{c(j)}(r); the (at most two) state vectors a block
// needs are staged in LDS.  NR right-hand sides (y + u ldy, t + u ldt) share the Psi loads.
template <typename PT, int NR>
__global__ __launch_bounds__(256) void k_spike_correct(int64_t n, int64_t ld, int K, int64_t s,
                                                       const PT* __restrict__ Psi, const cplx* __restrict__ t,
                                                       cplx* __restrict__ y, int64_t ldt, int64_t ldy,
                                                       const int* active) {
    if (active != nullptr && *active == 0) return;
    extern __shared__ cplx ts[];                     // NR x 2 K
    const int64_t jb = (int64_t)blockIdx.x * blockDim.x;
    const int64_t cb = jb / s;
    const int64_t ce = min(n - 1, jb + (int64_t)blockDim.x - 1) / s;
    for (int r = threadIdx.x; r < K; r += blockDim.x) {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            ts[u * 2 * K + r] = t[cb * K + r + u * ldt];
            ts[u * 2 * K + K + r] = t[ce * K + r + u * ldt];
        }
    }
    __syncthreads();
    const int64_t j = jb + threadIdx.x;
    if (j >= n) return;
    const int sel = (j / s == cb) ? 0 : K;
    cplx acc[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) acc[u] = y[j + u * ldy];
    const PT* pr = Psi + j;
    int r = 0;
    for (; r + 8 <= K; r += 8) {
        cplx v[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) v[w] = widen(pr[(int64_t)(r + w) * ld]);
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const cplx* tc = ts + u * 2 * K + sel;
#pragma unroll
            for (int w = 0; w < 8; ++w) acc[u] = fma_c(acc[u], v[w], tc[r + w]);
        }
    }
    for (; r < K; ++r) {
        const cplx v = widen(pr[(int64_t)r * ld]);
#pragma unroll
        for (int u = 0; u < NR; ++u) acc[u] = fma_c(acc[u], v, ts[u * 2 * K + sel + r]);
    }
#pragma unroll
    for (int u = 0; u < NR; ++u) y[j + u * ldy] = acc[u];
}

__global__ void k_fill_u32(unsigned* p, int count, unsigned v) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0ull;
}

// ipiv[j] = j past the matrix (identity extension to n16)
__global__ void k_pad_ipiv(int64_t n, int64_t n16, int* ipiv) {
    const int64_t j = n + threadIdx.x;
    if (j < n16) ipiv[j] = (int)j;
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

int threads_for(int rows) { return rows <= 256 ? 256 : (rows <= 512 ? 512 : 1024); }

// window (2 NR rows) + outputs (NR s) + inputs (s + 16) complex, and s pivots
size_t window_lds(int rows, int64_t s, int nr = 1) {
    return sizeof(cplx) * (2 * (size_t)nr * rows + (size_t)(nr + 1) * s + 16) + sizeof(int) * (size_t)s;
}

constexpr size_t LDS_LIMIT = 150 * 1024;   // as the chunk-length cap

// Zero-state sweeps (nrhs = 1) or the unit-state responses of all `nrhs` state rows,
// up to 4 of them per workgroup where the LDS allows it (the 1024-thread kernels, one).
template <typename Args>
simm_status launch_fwd(const Args& a, int64_t P, int nrhs, int W, int rows, int64_t s, hipStream_t st) {
    using GT = typename Args::storage;
    int nr = 1;
    if (nrhs > 1) {
        const int cap = (W <= 512) ? 4 : 1;
        for (int t = cap; t > 1; t /= 2)
            if (window_lds(rows, s, t) <= LDS_LIMIT) {
                nr = t;
                break;
            }
    }
    const size_t lds = window_lds(rows, s, nr);
    const dim3 grid((unsigned)P, (unsigned)((nrhs + nr - 1) / nr));
    if (W <= 256) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_fwd<256, 4, GT>), grid, dim3(256), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_fwd<256, 2, GT>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_fwd<256, 1, GT>), grid, dim3(256), lds, st, a);
    } else if (W <= 512) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_fwd<512, 4, GT>), grid, dim3(512), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_fwd<512, 2, GT>), grid, dim3(512), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_fwd<512, 1, GT>), grid, dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_chunk_fwd<1024, 1, GT>), grid, dim3(1024), lds, st, a);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}
template <typename Args>
simm_status launch_bwd(const Args& a, int64_t P, int nrhs, int W, int rows, int64_t s, hipStream_t st) {
    using GT = typename Args::storage;
    int nr = 1;
    if (nrhs > 1) {
        const int cap = (W <= 512) ? 4 : 1;
        for (int t = cap; t > 1; t /= 2)
            if (window_lds(rows, s, t) <= LDS_LIMIT) {
                nr = t;
                break;
            }
    }
    const size_t lds = window_lds(rows, s, nr);
    const dim3 grid((unsigned)P, (unsigned)((nrhs + nr - 1) / nr));
    if (W <= 256) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_bwd<256, 4, GT>), grid, dim3(256), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_bwd<256, 2, GT>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_bwd<256, 1, GT>), grid, dim3(256), lds, st, a);
    } else if (W <= 512) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_bwd<512, 4, GT>), grid, dim3(512), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_bwd<512, 2, GT>), grid, dim3(512), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_bwd<512, 1, GT>), grid, dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_chunk_bwd<1024, 1, GT>), grid, dim3(1024), lds, st, a);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// zero-state sweeps of nr columns: window (2 nr rows) + outputs (nr s) + inputs (nr (s + 16))
// complex, and s pivots
size_t window_lds0(int rows, int64_t s, int nr) {
    // several columns: outputs over inputs
    const size_t outs = nr > 1 ? 0 : (size_t)s;
    return sizeof(cplx) * (2 * (size_t)nr * rows + outs + (size_t)nr * (s + 16)) + sizeof(int) * (size_t)s;
}

template <typename Args>
simm_status launch_fwd0(const Args& a, int64_t P, int nr, int W, int rows, int64_t s, hipStream_t st) {
    using GT = typename Args::storage;
    const size_t lds = window_lds0(rows, s, nr);
    const dim3 grid((unsigned)P, 1u);
    if (W <= 256) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_fwd<256, 4, GT>), grid, dim3(256), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_fwd<256, 2, GT>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_fwd<256, 1, GT>), grid, dim3(256), lds, st, a);
    } else if (W <= 512) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_fwd<512, 4, GT>), grid, dim3(512), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_fwd<512, 2, GT>), grid, dim3(512), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_fwd<512, 1, GT>), grid, dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_chunk_fwd<1024, 1, GT>), grid, dim3(1024), lds, st, a);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}
template <typename Args>
simm_status launch_bwd0(const Args& a, int64_t P, int nr, int W, int rows, int64_t s, hipStream_t st) {
    using GT = typename Args::storage;
    const size_t lds = window_lds0(rows, s, nr);
    const dim3 grid((unsigned)P, 1u);
    if (W <= 256) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_bwd<256, 4, GT>), grid, dim3(256), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_bwd<256, 2, GT>), grid, dim3(256), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_bwd<256, 1, GT>), grid, dim3(256), lds, st, a);
    } else if (W <= 512) {
        if (nr == 4) hipLaunchKernelGGL((k_chunk_bwd<512, 4, GT>), grid, dim3(512), lds, st, a);
        else if (nr == 2) hipLaunchKernelGGL((k_chunk_bwd<512, 2, GT>), grid, dim3(512), lds, st, a);
        else hipLaunchKernelGGL((k_chunk_bwd<512, 1, GT>), grid, dim3(512), lds, st, a);
    } else {
        hipLaunchKernelGGL((k_chunk_bwd<1024, 1, GT>), grid, dim3(1024), lds, st, a);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace

int spike_max_nrhs(const SpikeFactor& f) {
    // the 1024-thread chunk kernels take one, chains of states longer than 512 one, and of
    // states longer than 256 two (more would spill registers)
    if (f.Wf > 512 || f.Wb > 512 || std::max(f.klx, f.K) > 32 * 16) return 1;
    const int cap = std::max(f.klx, f.K) > 16 * 16 ? 2 : 4;
    for (int nr = cap; nr > 1; nr /= 2)
        if (window_lds0(f.klx + 16, f.s, nr) <= LDS_LIMIT && window_lds0(f.K + 16, f.s, nr) <= LDS_LIMIT) return nr;
    return 1;
}

int64_t spike_chunk_len(int64_t n16, int kl, int K) {
    int64_t s = 0;
    if (const char* e = getenv("SIMM_SPIKE_CHUNK")) s = atoll(e);
    // balance the chunk sweeps (~s/16 panel steps of ~2 us) against the two-level chain
    // (~L + G steps of ~5-12 us) and the per-shift unit-state responses, whose fixed cost
    // per chunk grows with P: s ~ (3/8) sqrt(100 n) (n = 40,000 step medians with the
    // multi-vector unit-state responses: s = 500, 750, 1000, 1250 -> ~675, ~663, ~683,
    // ~700 ms)
    if (s <= 0) s = (int64_t)(std::sqrt((double)n16 * 100.0) * 0.375);
    // k_spike_correct stages the states of at most two chunks per 256-row block
    s = std::max<int64_t>(s, 256);
    s = std::max<int64_t>(s, std::max(kl, K) + 16);
    s = (s + 15) / 16 * 16;
    // a chunk's inputs, outputs and pivots are staged in LDS next to the window
    const int64_t rows = std::max(kl, K) + 16;
    const int64_t smax = ((150 * 1024 - 16 * (2 * rows + 16)) / (16 * 2 + 4)) / 16 * 16;
    s = std::min<int64_t>(s, smax);
    return std::min<int64_t>(s, n16);
}

// Transfer products of the two-level chain, chain order q (chunk q forward, P-1-q
// backward), for the groups g >= 1 (group g covers q0 = g L .. q1 - 1):
//     Pi_q = Phi_{q-1} ... Phi_{q0}  for q0 < q < q1,      PiFull_g = Phi_{q1-1} ... Phi_{q0}
// (the latter for the full groups 1 .. G-2 only: it carries the state to the next group).
// Phi, Pi are stored by rows ([i][r]); read as column-major arrays they are the
// transposes, so Pi_{q+1} = Phi_q Pi_q is the column-major product Pi_q^T Phi_q^T, formed
// for all groups at once by the batched FP64 matrix-core product.
static simm_status transfer_products(const SpikeFactor& f, bool forward, int K, const cplx* Phi, cplx* Pi,
                                     cplx* PiFull, hipStream_t st) {
    const int64_t KK = (int64_t)K * K, P = f.P, L = f.L, G = f.G;
    const int64_t len_last = P - (G - 1) * L;
    auto chunk = [&](int64_t q) { return forward ? q : P - 1 - q; };
    const int64_t sY = forward ? L * KK : -L * KK;
    // G > 1 implies L >= 2 (at least two chunks a group)
    for (int64_t d = 1; d <= L; ++d) {
        // groups 1 .. gmax take part in step d
        const int64_t gmax = (d < L) ? ((d < len_last) ? G - 1 : G - 2) : G - 2;
        if (gmax < 1) continue;
        const int64_t q = L + d - 1;   // group 1's q0 + d - 1
        if (d == 1) {
            const unsigned bx = (unsigned)std::min<int64_t>((KK + 255) / 256, 1024);
            hipLaunchKernelGGL(k_pi_first, dim3(bx, (unsigned)gmax), dim3(256), 0, st, K, P, L, forward ? 1 : 0, gmax,
                               Phi, Pi);
            SIMM_HIP_TRY(hipGetLastError());
            continue;
        }
        cplx* dst = (d < L) ? Pi + (L + d) * KK : PiFull + KK;
        const int64_t sX = (d < L) ? L * KK : KK;
        SIMM_TRY(project_batched(K, K, Pi + q * KK, K, L * KK, Phi + chunk(q) * KK, K, sY, K, dst, sX, (int)gmax, st));
    }
    return SIMM_OK;
}

// Per-panel blocks and unit-state responses of a factor stored in precision GT (the
// factor and its multipliers are read in the same precision, the arithmetic is FP64).
template <typename GT>
static simm_status prepare_blocks(SpikeFactor& f, const GT* LP, const GT* AB, GT* Gf, GT* Hb, GT* PsiL, GT* PsiU,
                                  hipStream_t st) {
    const int kl = f.klx, K = f.K;
    const int64_t n16 = f.n16;
    const unsigned npan = (unsigned)(n16 / 16);
    hipLaunchKernelGGL((k_blocks_fwd<GT, GT>), dim3(npan),
                       dim3(threads_for(kl + 16) <= 512 ? threads_for(kl + 16) : 512), 0, st, kl, LP, Gf);
    hipLaunchKernelGGL((k_blocks_bwd<GT, GT>), dim3(npan), dim3(threads_for(K + 16)), 0, st, f.n, K, f.kl + f.ku,
                       2 * f.kl + f.ku + 1, AB, Hb);
    SIMM_HIP_TRY(hipGetLastError());
    SpikeFwdT<GT> a{};
    a.n = f.n;
    a.n16 = n16;
    a.kl = kl;
    a.ipiv = f.ipiv;
    a.G = Gf;
    a.s = f.s;
    a.mode = 1;
    a.Psi = PsiL;
    a.Phi = f.PhiL;
    SIMM_TRY(launch_fwd(a, f.P, kl, f.Wf, kl + 16, f.s, st));
    SpikeBwdT<GT> b{};
    b.n = f.n;
    b.n16 = n16;
    b.K = K;
    b.H = Hb;
    b.s = f.s;
    b.mode = 1;
    b.Psi = PsiU;
    b.Phi = f.PhiU;
    SIMM_TRY(launch_bwd(b, f.P, K, f.Wb, K + 16, f.s, st));
    return SIMM_OK;
}

simm_status spike_prepare(SpikeFactor& f, hipStream_t st) {
    f.n16 = (f.n + 15) / 16 * 16;
    if (f.n16 > f.n) hipLaunchKernelGGL(k_pad_ipiv, dim3(1), dim3(16), 0, st, f.n, f.n16, f.ipiv);
    // effective upper bandwidth of U: ku plus the largest interchange distance
    int* d_jump = nullptr;
    SIMM_HIP_TRY(hipMallocAsync((void**)&d_jump, sizeof(int), st));
    hipLaunchKernelGGL(k_max_jump, dim3(1), dim3(256), 0, st, f.n, (const int*)f.ipiv, d_jump);
    int jump = 0;
    SIMM_HIP_TRY(hipMemcpyAsync(&jump, d_jump, sizeof(int), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    SIMM_HIP_TRY(hipFreeAsync(d_jump, st));
    f.K = (int)std::min<int64_t>(std::min<int64_t>(f.kl + f.ku, f.ku + std::max(0, jump)), f.n - 1);
    f.K = std::max(f.K, 1);
    f.klx = std::max(1, (int)std::min<int64_t>(f.kl, f.n - 1));
    if (f.n > (int64_t)1 << 30) {
        set_error("order above 2^30 is not supported by the partitioned sweeps");
        return SIMM_EUNSUPPORTED;
    }
    if (f.klx + 16 > 1024 || f.K + 16 > 1024) {
        set_error("band too wide for the partitioned sweeps (bandwidth + 16 > 1024)");
        return SIMM_EUNSUPPORTED;
    }
    f.s = spike_chunk_len(f.n16, f.klx, f.K);
    f.P = (f.n16 + f.s - 1) / f.s;
    // groups of the two-level chain: ~(2/3) sqrt(P) groups (concurrent groups slow each
    // other's steps, so somewhat fewer and longer groups than the sqrt(P) that balances
    // the step counts), at least 2 chunks a group (SIMM_SPIKE_GROUPS overrides; 1 = one
    // chain over all chunks)
    {
        int64_t G = (f.P >= 8) ? std::max<int64_t>(1, std::lround(std::sqrt((double)f.P) * 2.0 / 3.0)) : 1;
        if (const char* e = getenv("SIMM_SPIKE_GROUPS")) G = std::max<int64_t>(1, atoll(e));
        G = std::min<int64_t>(G, std::max<int64_t>(1, f.P / 2));
        f.L = (f.P + G - 1) / G;
        f.G = (f.P + f.L - 1) / f.L;
    }
    f.Wf = threads_for(f.klx + 16);
    f.Wb = threads_for(f.K + 16);
    const int kl = f.klx, K = f.K;
    const int64_t n16 = f.n16;
    const size_t two = f.G > 1 ? 1 : 0;    // transfer products only with more than one group
    // n-sized per-panel blocks and unit-state responses, in the factor's precision
    const size_t big = (size_t)n16 * (kl + 16) + (size_t)n16 * (K + 16) + (size_t)n16 * kl + (size_t)n16 * K;
    const size_t esz = f.f32 ? sizeof(cplxf) : sizeof(cplx);
    const size_t elems = (size_t)f.P * kl * kl + (size_t)f.P * K * K + (size_t)f.P * kl * 2 + (size_t)f.P * K * 2 +
                         (size_t)n16 + two * ((size_t)(f.P + f.G) * ((size_t)kl * kl + (size_t)K * K)) +
                         (size_t)f.G * 2 * (kl + K) + (size_t)(f.G + 1) * 16 + 64;
    SIMM_HIP_TRY(device_malloc(&f.mem, sizeof(cplx) * elems + esz * big + 20 * 256));
    char* p = reinterpret_cast<char*>(f.mem);
    auto take_b = [&](size_t bytes) {
        char* r = p;
        p += (bytes + 255) & ~(size_t)255;
        return r;
    };
    auto take = [&](size_t count) { return reinterpret_cast<cplx*>(take_b(sizeof(cplx) * count)); };
    if (f.f32) {
        auto take_f = [&](size_t count) { return reinterpret_cast<cplxf*>(take_b(sizeof(cplxf) * count)); };
        f.Gf32 = take_f((size_t)n16 * (kl + 16));
        f.Hb32 = take_f((size_t)n16 * (K + 16));
        f.PsiL32 = take_f((size_t)n16 * kl);
        f.PsiU32 = take_f((size_t)n16 * K);
    } else {
        f.Gf = take((size_t)n16 * (kl + 16));
        f.Hb = take((size_t)n16 * (K + 16));
        f.PsiL = take((size_t)n16 * kl);
        f.PsiU = take((size_t)n16 * K);
    }
    f.PhiL = take((size_t)f.P * kl * kl);
    f.PhiU = take((size_t)f.P * K * K);
    f.tauL = take((size_t)f.P * kl);
    f.tL = take((size_t)f.P * kl);
    f.tauU = take((size_t)f.P * K);
    f.tU = take((size_t)f.P * K);
    f.z = take((size_t)n16);
    if (f.G > 1) {
        f.PiL = take((size_t)f.P * kl * kl);
        f.PiU = take((size_t)f.P * K * K);
        f.PiFullL = take((size_t)f.G * kl * kl);
        f.PiFullU = take((size_t)f.G * K * K);
    }
    f.goutL = take((size_t)f.G * kl);
    f.goutU = take((size_t)f.G * K);
    f.tgL = take((size_t)f.G * kl);
    f.tgU = take((size_t)f.G * K);
    // one barrier counter per group and one for the chain over groups, each on a line of
    // its own (spinning workgroups of different groups must not share a cache line)
    f.counter = reinterpret_cast<unsigned*>(take((size_t)(f.G + 1) * (SPIKE_CTR_STRIDE / 4)));
    f.err = reinterpret_cast<int*>(take(4));
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(f.err), 1, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, f.counter, (int)((f.G + 1) * SPIKE_CTR_STRIDE), 0u);
    if (f.f32) SIMM_TRY(prepare_blocks<cplxf>(f, f.LP32, f.AB32, f.Gf32, f.Hb32, f.PsiL32, f.PsiU32, st));
    else SIMM_TRY(prepare_blocks<cplx>(f, f.LP, f.AB, f.Gf, f.Hb, f.PsiL, f.PsiU, st));
    if (f.G > 1) {
        SIMM_TRY(transfer_products(f, true, kl, f.PhiL, f.PiL, f.PiFullL, st));
        SIMM_TRY(transfer_products(f, false, K, f.PhiU, f.PiU, f.PiFullU, st));
    }
    // a partitioned factor: its spikes and reduced system, from D's sweeps
    if (f.bs > 0) SIMM_TRY(part_prepare(f, st));
    return SIMM_OK;
}

// A second set of the per-application buffers of a prepared factor (sweep outputs,
// chain states, group outputs, barrier counters, error flag), so that applications of
// one factor can run on several streams at once.  The clone shares the factor data
// and spike_release on it frees only its own buffers.
simm_status spike_clone_scratch(const SpikeFactor& base, SpikeFactor& out, hipStream_t st, bool ordered, int nrhs) {
    out = base;
    out.mem = nullptr;
    out.part_mem = nullptr;   // spikes and reduced inverse stay the base's
    nrhs = std::max(1, nrhs);
    out.nrhs = nrhs;
    const int kl = base.klx, K = base.K;
    const size_t part = base.bs > 0 ? (size_t)base.n16 * nrhs + (size_t)base.nr + 32 : 0;
    const size_t elems = ((size_t)base.n16 + (size_t)base.P * kl * 2 + (size_t)base.P * K * 2 +
                          (size_t)base.G * 2 * (kl + K)) * (size_t)nrhs + (size_t)(base.G + 1) * 16 + 64 + part;
    if (ordered) SIMM_HIP_TRY(device_malloc_async(&out.mem, sizeof(cplx) * elems + 14 * 256, st));
    else SIMM_HIP_TRY(device_malloc(&out.mem, sizeof(cplx) * elems + 14 * 256));
    char* p = reinterpret_cast<char*>(out.mem);
    auto take = [&](size_t count) {
        char* r = p;
        p += (sizeof(cplx) * count + 255) & ~(size_t)255;
        return reinterpret_cast<cplx*>(r);
    };
    // nrhs slabs each, at the strides apply_t uses
    out.tauL = take((size_t)base.P * kl * nrhs);
    out.tL = take((size_t)base.P * kl * nrhs);
    out.tauU = take((size_t)base.P * K * nrhs);
    out.tU = take((size_t)base.P * K * nrhs);
    out.z = take((size_t)base.n16 * nrhs);
    out.goutL = take((size_t)base.G * kl * nrhs);
    out.goutU = take((size_t)base.G * K * nrhs);
    out.tgL = take((size_t)base.G * kl * nrhs);
    out.tgU = take((size_t)base.G * K * nrhs);
    out.counter = reinterpret_cast<unsigned*>(take((size_t)(base.G + 1) * (SPIKE_CTR_STRIDE / 4)));
    out.err = reinterpret_cast<int*>(take(4));
    if (base.bs > 0) {
        out.pg = take((size_t)base.n16 * nrhs);
        out.pz = take((size_t)base.nr * nrhs);
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(out.err), 1, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, out.counter, (int)((base.G + 1) * SPIKE_CTR_STRIDE), 0u);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

void spike_release_ordered(SpikeFactor& f, hipStream_t st) {
    if (f.mem) (void)hipFreeAsync(f.mem, st);
    f.mem = nullptr;
}

void spike_release(SpikeFactor& f) {
    (void)hipFree(f.mem);
    (void)hipFree(f.part_mem);
    f.mem = nullptr;
    f.part_mem = nullptr;
}

// Chains of concurrent applications share the device.  A chain's workgroups spin at
// device-scope barriers until all of a group's run, so chains on several streams whose
// workgroups together exceed what the compute units hold could each wait for slots the
// others' spinning workgroups keep (a bounded spin then reports the chain as timed
// out).  Every phase that launches chains (a Krylov phase, the spike solves, a single
// application) therefore holds, from before its first chain until its stream is done,
// a share of a per-device budget of 256 compute units: a chain workgroup takes a
// compute unit's registers for the 32- and 64-row forms (one wave per SIMD), half of
// them for the 16-row form.  Only chains spin; every other kernel's workgroups leave.
// A phase asking for more than the budget runs alone (a chain alone always progresses:
// its groups are dispatched in order and wait only on themselves).
namespace {
constexpr int kChainBudget = 512;   // half compute units
struct ChainBudget {
    std::mutex mu;
    std::condition_variable cv;
    int avail = kChainBudget;
};
std::mutex g_budgets_mu;
std::map<int, std::unique_ptr<ChainBudget>> g_budgets;
ChainBudget* chain_budget(int dev) {
    std::lock_guard<std::mutex> lk(g_budgets_mu);
    auto& b = g_budgets[dev];
    if (!b) b = std::make_unique<ChainBudget>();
    return b.get();
}
}  // namespace

int spike_chain_weight(const SpikeFactor& f) {
    auto w = [&](int K) { return ((K + 15) / 16) * (int)std::max<int64_t>(1, f.G) * (K <= 16 * 16 ? 1 : 2); };
    return std::max(1, std::min(kChainBudget, std::max(w(f.klx), w(f.K))));
}

int spike_chain_budget() { return kChainBudget; }

simm_status ChainSlots::acquire(int weight, hipStream_t s) {
    release();
    weight = std::max(1, std::min(kChainBudget, weight));
    SIMM_HIP_TRY(hipGetDevice(&dev));
    ChainBudget* b = chain_budget(dev);
    std::unique_lock<std::mutex> lk(b->mu);
    b->cv.wait(lk, [&]() { return b->avail >= weight; });
    b->avail -= weight;
    w = weight;
    st = s;
    return SIMM_OK;
}

void ChainSlots::release() {
    if (w <= 0) return;
    (void)hipStreamSynchronize(st);   // the phase's chains are done
    ChainBudget* b = chain_budget(dev);
    {
        std::lock_guard<std::mutex> lk(b->mu);
        b->avail += w;
    }
    b->cv.notify_all();
    w = 0;
}

// One chain launch: `groups` groups of L chunks (chain order) over P chunks, each group
// with its own barrier counter.
static simm_status run_chain(const SpikeFactor& f, bool forward, int K, int64_t P, int64_t L, int64_t groups,
                             const cplx* Phi, const cplx* tau, cplx* tstate, cplx* gout, const cplx* init_src,
                             int64_t init_row0, int64_t n, unsigned* counter, const int* active, hipStream_t st,
                             int nr = 1, int64_t ldt = 0, int64_t ldg = 0, int64_t ldi = 0) {
    SpikeChain c{};
    c.ldt = ldt;
    c.ldg = ldg;
    c.ldi = ldi;
    c.n = n;
    c.K = K;
    c.P = P;
    c.L = L;
    c.forward = forward ? 1 : 0;
    c.Phi = Phi;
    c.tau = tau;
    c.t = tstate;
    c.gout = gout;
    c.init_src = init_src;
    c.init_row0 = init_row0;
    c.counter = counter;
    c.err = f.err;
    c.active = active;
    // 16 threads per state row, 16 rows per workgroup: more, smaller workgroups make
    // the device-scope barrier of every step dearer than the rows they save
    const dim3 grid((unsigned)((K + 15) / 16), (unsigned)groups);
    if ((nr > 1 && K > 32 * 16) || (nr > 2 && K > 16 * 16)) {
        set_error("several right-hand sides: four need chain states of at most 256, two of at most 512");
        return SIMM_EINVAL;
    }
    if (nr == 4) {
        hipLaunchKernelGGL((k_spike_chain<16, 16, 4>), grid, dim3(CH_THREADS), 0, st, c);
    } else if (nr == 2) {
        if (K <= 16 * 16) hipLaunchKernelGGL((k_spike_chain<16, 16, 2>), grid, dim3(CH_THREADS), 0, st, c);
        else hipLaunchKernelGGL((k_spike_chain<32, 16, 2>), grid, dim3(CH_THREADS), 0, st, c);
    } else {
        if (K <= 16 * 16) hipLaunchKernelGGL((k_spike_chain<16, 16, 1>), grid, dim3(CH_THREADS), 0, st, c);
        else if (K <= 32 * 16) hipLaunchKernelGGL((k_spike_chain<32, 16, 1>), grid, dim3(CH_THREADS), 0, st, c);
        else hipLaunchKernelGGL((k_spike_chain<64, 16, 1>), grid, dim3(CH_THREADS), 0, st, c);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// The chain over the chunks' boundary states of one sweep direction: one level, or
// groups in parallel, the chain over the groups' start states and the fix-up.
// nr right-hand sides: slabs of t and tau every P K, of gout and tg every G K, of the
// initial states every ldi.
static simm_status chain_states(const SpikeFactor& f, bool forward, int K, const cplx* Phi, const cplx* tau, cplx* t,
                                const cplx* Pi, const cplx* PiFull, cplx* gout, cplx* tg, const cplx* init_src,
                                int64_t init_row0, const int* active, hipStream_t st, int nr = 1, int64_t ldi = 0) {
    const int64_t ldt = f.P * K, ldg = f.G * K;
    // the counters are zero here: zeroed when the sweep data was made, and every chain
    // launch leaves its group's counters at zero when it ends
    SIMM_TRY(run_chain(f, forward, K, f.P, f.L, f.G, Phi, tau, t, gout, init_src, init_row0, f.n, f.counter, active,
                       st, nr, ldt, ldg, ldi));
    if (f.G == 1) return SIMM_OK;
    // T_1 = gout_0; T_{g+1} = gout_g + PiFull_g T_g (g = 1 .. G-2), into tg[g-1]
    const int64_t KK = (int64_t)K * K;
    SIMM_TRY(run_chain(f, true, K, f.G - 1, f.G - 1, 1, PiFull + KK, gout + K, tg, nullptr, gout, 0, K,
                       f.counter + f.G * SPIKE_CTR_STRIDE, active, st, nr, ldg, 0, ldg));
    const dim3 grid((unsigned)((K + 15) / 16), (unsigned)f.P);
    const int fw = forward ? 1 : 0;
    if (nr == 4) {   // K <= 256, and K <= 512 for two (checked by run_chain)
        hipLaunchKernelGGL((k_spike_fix<16, 4>), grid, dim3(256), 0, st, K, f.P, f.L, fw, Pi, tg, t, ldg, ldt, active);
    } else if (nr == 2) {
        if (K <= 16 * 16) hipLaunchKernelGGL((k_spike_fix<16, 2>), grid, dim3(256), 0, st, K, f.P, f.L, fw, Pi, tg, t, ldg,
                                             ldt, active);
        else hipLaunchKernelGGL((k_spike_fix<32, 2>), grid, dim3(256), 0, st, K, f.P, f.L, fw, Pi, tg, t, ldg, ldt, active);
    } else {
        if (K <= 16 * 16) hipLaunchKernelGGL((k_spike_fix<16, 1>), grid, dim3(256), 0, st, K, f.P, f.L, fw, Pi, tg, t, ldg,
                                             ldt, active);
        else if (K <= 32 * 16) hipLaunchKernelGGL((k_spike_fix<32, 1>), grid, dim3(256), 0, st, K, f.P, f.L, fw, Pi, tg, t,
                                                  ldg, ldt, active);
        else hipLaunchKernelGGL((k_spike_fix<64, 1>), grid, dim3(256), 0, st, K, f.P, f.L, fw, Pi, tg, t, ldg, ldt, active);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

template <typename GT, int NR>
void launch_correct(const SpikeFactor& f, int K, const GT* Psi, const cplx* t, cplx* y, int64_t ldy, const int* active,
                    hipStream_t st) {
    const unsigned blocks = (unsigned)((f.n + 255) / 256);
    hipLaunchKernelGGL((k_spike_correct<GT, NR>), dim3(blocks), dim3(256), sizeof(cplx) * 2 * K * NR, st, f.n, f.n16, K,
                       f.s, Psi, t, y, f.P * (int64_t)K, ldy, active);
}

// nr columns u + r ldu -> y + r ldy (nr = 1: ldu, ldy unused); the scratch holds f.nrhs slabs.
template <typename GT>
static simm_status apply_t(const SpikeFactor& f, const GT* Gf, const GT* Hb, const GT* PsiL, const GT* PsiU,
                           const cplx* u, cplx* y, const int* active, hipStream_t st, int nr = 1, int64_t ldu = 0,
                           int64_t ldy = 0) {
    auto correct = [&](int K, const GT* Psi, const cplx* t, cplx* out, int64_t ld) {
        if (nr == 4) launch_correct<GT, 4>(f, K, Psi, t, out, ld, active, st);
        else if (nr == 2) launch_correct<GT, 2>(f, K, Psi, t, out, ld, active, st);
        else launch_correct<GT, 1>(f, K, Psi, t, out, ld, active, st);
    };
    // forward: z = L^{-1} P u
    cplx* z = f.z;
    SpikeFwdT<GT> a{};
    a.n = f.n;
    a.n16 = f.n16;
    a.kl = f.klx;
    a.ipiv = f.ipiv;
    a.G = Gf;
    a.s = f.s;
    a.mode = 0;
    a.u = u;
    a.y = z;
    a.tau = f.tauL;
    a.active = active;
    a.ldu = ldu;
    a.ldy = f.n16;
    a.ldt = f.P * (int64_t)f.klx;
    SIMM_TRY(launch_fwd0(a, f.P, nr, f.Wf, f.klx + 16, f.s, st));
    SIMM_TRY(chain_states(f, true, f.klx, f.PhiL, f.tauL, f.tL, f.PiL, f.PiFullL, f.goutL, f.tgL, u, 0, active, st, nr,
                          ldu));
    correct(f.klx, PsiL, f.tL, z, f.n16);
    // backward: y = U^{-1} z
    SpikeBwdT<GT> b{};
    b.n = f.n;
    b.n16 = f.n16;
    b.K = f.K;
    b.H = Hb;
    b.s = f.s;
    b.mode = 0;
    b.z = z;
    b.y = y;
    b.tau = f.tauU;
    b.active = active;
    b.ldu = f.n16;
    b.ldy = ldy;
    b.ldt = f.P * (int64_t)f.K;
    SIMM_TRY(launch_bwd0(b, f.P, nr, f.Wb, f.K + 16, f.s, st));
    SIMM_TRY(chain_states(f, false, f.K, f.PhiU, f.tauU, f.tU, f.PiU, f.PiFullU, f.goutU, f.tgU, z, f.n16 - f.K, active,
                          st, nr, f.n16));
    correct(f.K, PsiU, f.tU, y, ldy);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status spike_apply_diag(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st) {
    if (f.f32) return apply_t<cplxf>(f, f.Gf32, f.Hb32, f.PsiL32, f.PsiU32, u, y, active, st);
    return apply_t<cplx>(f, f.Gf, f.Hb, f.PsiL, f.PsiU, u, y, active, st);
}

simm_status spike_apply_diag_nr(const SpikeFactor& f, const cplx* u, int64_t ldu, cplx* y, int64_t ldy, int nr,
                                hipStream_t st) {
    if (!(nr == 1 || nr == 2 || nr == 4) || nr > f.nrhs || nr > spike_max_nrhs(f)) {
        set_error("right-hand sides per application: 1, 2 or 4, within the scratch and the chunk kernels' LDS");
        return SIMM_EINVAL;
    }
    if (f.f32) return apply_t<cplxf>(f, f.Gf32, f.Hb32, f.PsiL32, f.PsiU32, u, y, nullptr, st, nr, ldu, ldy);
    return apply_t<cplx>(f, f.Gf, f.Hb, f.PsiL, f.PsiU, u, y, nullptr, st, nr, ldu, ldy);
}

simm_status spike_apply_nr(const SpikeFactor& f, const cplx* u, int64_t ldu, cplx* y, int64_t ldy, int nr,
                           hipStream_t st) {
    if (f.bs > 0) return part_apply_nr(f, u, ldu, y, ldy, nr, st);
    return spike_apply_diag_nr(f, u, ldu, y, ldy, nr, st);
}

simm_status spike_apply(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st) {
    if (f.bs > 0) return part_apply(f, u, y, active, st);
    return spike_apply_diag(f, u, y, active, st);
}

int64_t spike_bytes_per_apply(const SpikeFactor& f) {
    // algorithmic bytes: each stored factor entry within the effective band read once,
    // input read once, output written once
    int64_t lower = 0, upper = 0;
    for (int64_t j = 0; j < f.n; ++j) {
        lower += std::min<int64_t>(f.kl, f.n - 1 - j);
        upper += std::min<int64_t>(f.K, j) + 1;
    }
    // a partitioned factor: its spikes and the reduced inverse once more
    const int64_t part = f.bs > 0 ? f.n * (int64_t)(f.pkl + f.pku) + f.nr * f.nr : 0;
    return 16 * (lower + upper + 2 * f.n + part);
}

}  // namespace simm
