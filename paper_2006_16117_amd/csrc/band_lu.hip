// Shifted pencil assembly and banded LU with partial pivoting (gfx950).
//
// The Cayley transform of Sec. 2 needs one factorization of A - sigma B per shift
// (sigma not an eigenvalue).  The factor uses LAPACK general-band LU storage:
// ldab = 2 kl + ku + 1 rows, kv = kl + ku; U(i,j) at row kv + i - j (kv super-
// diagonals after fill), the multipliers of column j at rows kv+1 .. kv+kl.  As in
// LAPACK's band LU, the row interchange of step j is applied to columns >= j
// only, so column j keeps its multipliers as computed ("interleaved" L) and a
// solve applies interchange and elimination column by column.
//
// Blocked right-looking schedule, one launch per panel of NB columns:
//   launch b:  every workgroup takes a slice of the columns right of panel b,
//              applies panel b's interchanges, the unit-lower triangular solve and
//              the rank-NB update (trailing window = rows of the panel + kl), and
//              workgroup 0, which owns panel b+1, then factors panel b+1 in LDS.
// Consecutive launches on one stream order the panels; no workgroup ever waits
// on another.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

// a1: C = A - sigma B written into LU band storage (fill rows zeroed).
__global__ void k_assemble_shifted(int64_t n, int kl, int ku, const cplx* __restrict__ A, int kla, int kua,
                                   const cplx* __restrict__ B, int klb, int kub, cplx sigma,
                                   cplx* __restrict__ AB) {
    const int kv = kl + ku, ldab = 2 * kl + ku + 1;
    const int64_t c = blockIdx.x;
    for (int r = threadIdx.x; r < ldab; r += blockDim.x) {
        const int d = r - kv;          // i - c
        const int64_t i = c + d;
        cplx v = mk(0.0, 0.0);
        if (i >= 0 && i < n) {
            if (d >= -kua && d <= kla) v = A[(int64_t)(kua + d) + c * (kla + kua + 1)];
            if (B) {
                if (d >= -kub && d <= klb) v = v - sigma * B[(int64_t)(kub + d) + c * (klb + kub + 1)];
            } else if (d == 0) {
                v = v - sigma;
            }
        }
        AB[(int64_t)r + c * ldab] = v;
    }
}

namespace {

constexpr int LU_THREADS = 256;

__host__ __device__ inline int lds_ld(int rows) { return ((rows + 15) / 16) * 16 + 1; }

struct LuArgs {
    int64_t n;
    int kl, ku, kv, ldab;
    int nb;          // panel width
    int cw;          // columns per trailing workgroup
    cplx* AB;
    int* ipiv;       // 0-based global row of the pivot of each column
    cplx* lt[2];     // permuted panel multipliers, (nb + kl) x nb column-major, double buffered
    int* info;       // first singular column + 1 (INT_MAX if none)
    int64_t zidx;    // index of the zero entry stored after the band
};

// Index of band entry (i, c), or of the zero entry when (i, c) lies outside the
// band: loads through it are unconditional, so a loop of them keeps many in flight.
__device__ inline int64_t ab_idx(const LuArgs& a, int64_t i, int64_t c) {
    const int64_t d = i - c;
    const bool in = i >= 0 && i < a.n && c >= 0 && c < a.n && d >= -a.kv && d <= a.kl;
    return in ? (int64_t)(a.kv + d) + c * a.ldab : a.zidx;
}

// dst[r + c*ldd] = band(i0 + r, c0 + c) for rfrom <= r < R, c < C (C <= 16): one row per
// thread, its 16 column loads issued together.
__device__ inline void load_tile(const LuArgs& a, cplx* dst, int ldd, int64_t i0, int64_t c0, int R, int C, int rfrom) {
    for (int r = rfrom + (int)threadIdx.x; r < R; r += LU_THREADS) {
        cplx v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = a.AB[c < C ? ab_idx(a, i0 + r, c0 + c) : a.zidx];
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < C) dst[r + c * ldd] = v[c];
    }
}

__device__ inline cplx ab_get(const LuArgs& a, int64_t i, int64_t c) {
    const int64_t d = i - c;
    if (i < 0 || i >= a.n || c < 0 || c >= a.n || d < -a.kv || d > a.kl) return mk(0.0, 0.0);
    return a.AB[(int64_t)(a.kv + d) + c * a.ldab];
}
__device__ inline void ab_put(const LuArgs& a, int64_t i, int64_t c, cplx v) {
    const int64_t d = i - c;
    if (i < 0 || i >= a.n || c < 0 || c >= a.n || d < -a.kv || d > a.kl) return;
    a.AB[(int64_t)(a.kv + d) + c * a.ldab] = v;
}

// Factor the panel held in P (rows j1 .. j1+R1-1, columns j1 .. j1+nb1-1, leading
// dimension ldp) in place; store multipliers / U / pivots in the band and the
// permuted multipliers in `lt_out`.  Interchanges are applied to every panel
// column (so P ends up with the permuted multipliers a blocked update needs);
// the band keeps each column's multipliers as they were when computed, which is
// recovered at the end by undoing the later interchanges on that column.
__device__ void factor_panel(const LuArgs& a, cplx* P, int ldp, int64_t j1, int nb1, int R1, cplx* lt_out,
                             double* red_v, int* red_i, int* piv_s) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int t = 0; t < nb1; ++t) {
        const int64_t j = j1 + t;
        const int km = (int)min((int64_t)a.kl, a.n - 1 - j);
        // pivot search: first index of max |re| + |im| over rows t .. t+km
        double best = -1.0;
        int bidx = t + km + 1;
        for (int r = t + tid; r <= t + km; r += LU_THREADS) {
            const double v = cabs1(P[r + t * ldp]);
            if (v > best) { best = v; bidx = r; }
        }
#pragma unroll
        for (int msk = 32; msk >= 1; msk >>= 1) {
            const double v2 = __shfl_xor(best, msk, 64);
            const int i2 = __shfl_xor(bidx, msk, 64);
            if (v2 > best || (v2 == best && i2 < bidx)) { best = v2; bidx = i2; }
        }
        if (lane == 0) {
            red_v[wave] = best;
            red_i[wave] = bidx;
        }
        lds_barrier();
        best = red_v[0];
        bidx = red_i[0];
        for (int w = 1; w < LU_THREADS / 64; ++w) {
            if (red_v[w] > best || (red_v[w] == best && red_i[w] < bidx)) { best = red_v[w]; bidx = red_i[w]; }
        }
        const int rp = bidx;
        const bool zero = !(best > 0.0);
        if (tid == 0) {
            a.ipiv[j] = (int)(j1 + rp);
            piv_s[t] = zero ? t : rp;
        }
        if (zero) {
            if (tid == 0) atomicMin(a.info, (int)(j + 1));
            // LAPACK semantics: record the pivot, no interchange or elimination.
            lds_barrier();
            continue;
        }
        if (rp != t) {
            for (int c = tid; c < nb1; c += LU_THREADS) {
                cplx tmp = P[t + c * ldp];
                P[t + c * ldp] = P[rp + c * ldp];
                P[rp + c * ldp] = tmp;
            }
        }
        lds_barrier();
        const cplx piv = P[t + t * ldp];
        for (int r = t + 1 + tid; r <= t + km; r += LU_THREADS) P[r + t * ldp] = cdiv(P[r + t * ldp], piv);
        lds_barrier();
        // rank-1 update: thread -> column t+1 + (tid % 16), rows t+1 + tid/16 + 16k
        {
            const int c = t + 1 + (tid & 15);
            if (c < nb1) {
                const cplx ptc = P[t + c * ldp];
                for (int r = t + 1 + (tid >> 4); r <= t + km; r += LU_THREADS / 16)
                    P[r + c * ldp] = fms(P[r + c * ldp], P[r + t * ldp], ptc);
            }
        }
        lds_barrier();
    }
    // permuted multipliers and U for the trailing update of the next launch; U to the band
    for (int t = 0; t < nb1; ++t) {
        for (int r = tid; r < R1; r += LU_THREADS) {
            const cplx v = P[r + t * ldp];
            if (r <= t) ab_put(a, j1 + r, j1 + t, v);
            lt_out[r + t * (a.nb + a.kl)] = v;
        }
    }
    lds_barrier();
    // undo the interchanges of later steps on each column's multipliers, then store them
    for (int t = tid; t < nb1; t += LU_THREADS) {
        for (int t2 = nb1 - 1; t2 > t; --t2) {
            const int p2 = piv_s[t2];
            if (p2 != t2) {
                cplx tmp = P[t2 + t * ldp];
                P[t2 + t * ldp] = P[p2 + t * ldp];
                P[p2 + t * ldp] = tmp;
            }
        }
    }
    lds_barrier();
    for (int t = 0; t < nb1; ++t) {
        for (int r = t + 1 + tid; r <= t + a.kl && r < R1; r += LU_THREADS) ab_put(a, j1 + r, j1 + t, P[r + t * ldp]);
    }
}

}  // namespace

__global__ __launch_bounds__(LU_THREADS) void k_band_lu_step(LuArgs a, int64_t b) {
    extern __shared__ cplx smem[];
    __shared__ double red_v[LU_THREADS / 64];
    __shared__ int red_i[LU_THREADS / 64];
    __shared__ int piv_s[32];
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;
    const int nb = a.nb;
    // LDS leading dimensions padded to 1 (mod 16) complex entries, so the 16 columns a
    // wavefront touches start in 16 different banks
    const int ldl = lds_ld(nb + a.kl);         // rows of the panel buffer
    cplx* Pan = smem;                          // ldl x nb      : permuted multipliers of panel b
    const int ldx = lds_ld(2 * nb + a.kl);
    cplx* Xc = smem + (size_t)ldl * nb;        // ldx x ncols   : my column slice, rows j0 ..

    const int64_t j0 = b * nb;                                  // panel b (b may be -1)
    const int nbp = (b >= 0) ? (int)min((int64_t)nb, a.n - j0) : 0;
    const int64_t j1 = (b >= 0) ? j0 + nbp : 0;                 // panel b+1
    const int nb1 = (int)max((int64_t)0, min((int64_t)nb, a.n - j1));

    // my column slice
    int64_t c0, c1;
    if (wg == 0) {
        c0 = j1;
        c1 = j1 + nb1;
    } else {
        if (b < 0) return;
        const int64_t jmax = min(a.n - 1, j0 + nbp - 1 + (int64_t)a.kv);
        c0 = j1 + nb1 + (int64_t)(wg - 1) * a.cw;
        c1 = min(c0 + a.cw, jmax + 1);
        if (c0 > jmax) return;
    }
    const int ncols = (int)(c1 - c0);

    if (b >= 0 && ncols > 0) {
        const int Rb = (int)min((int64_t)(nbp + a.kl), a.n - j0);   // rows j0 .. j0+Rb-1 touched
        const cplx* lt_in = a.lt[b & 1];
        {
            const int ldg = a.nb + a.kl;        // leading dimension of the global panel buffer
            for (int r = tid; r < Rb; r += LU_THREADS) {
                cplx v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) v[q] = lt_in[r + (q < nbp ? q : 0) * ldg];
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (q < nbp) Pan[r + q * ldl] = v[q];
            }
        }
        load_tile(a, Xc, ldx, j0, c0, Rb, ncols, 0);
        if (tid < nbp) piv_s[tid] = (int)(a.ipiv[j0 + tid] - j0);
        lds_barrier();
        // interchanges, in order (one thread per column)
        for (int c = tid; c < ncols; c += LU_THREADS) {
            for (int t = 0; t < nbp; ++t) {
                const int p = piv_s[t];
                if (p != t) {
                    cplx tmp = Xc[t + c * ldx];
                    Xc[t + c * ldx] = Xc[p + c * ldx];
                    Xc[p + c * ldx] = tmp;
                }
            }
        }
        lds_barrier();
        // unit lower triangular solve: thread (column tid % 16, row tid / 16), one step per t
        {
            const int c = tid & 15, rr = tid >> 4;
            for (int t = 0; t + 1 < nbp; ++t) {
                if (c < ncols && rr > t && rr < nbp)
                    Xc[rr + c * ldx] = fms(Xc[rr + c * ldx], Pan[rr + t * ldl], Xc[t + c * ldx]);
                lds_barrier();
            }
        }
        // rank-nbp update of rows nbp .. Rb-1: thread -> column tid % 16 (its U column in
        // registers), rows nbp + tid/16 + 16k
        {
            const int c = tid & 15;
            if (c < ncols) {
                cplx u[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) u[q] = (q < nbp) ? Xc[q + c * ldx] : mk(0.0, 0.0);
                for (int r = nbp + (tid >> 4); r < Rb; r += LU_THREADS / 16) {
                    cplx acc = Xc[r + c * ldx];
#pragma unroll
                    for (int q = 0; q < 16; ++q)
                        if (q < nbp) acc = fms(acc, Pan[r + q * ldl], u[q]);
                    Xc[r + c * ldx] = acc;
                }
            }
        }
        lds_barrier();
        // write back; workgroup 0 keeps rows j1.. in LDS for its panel
        {
            const int rend = (wg != 0) ? Rb : nbp;
            for (int c = 0; c < ncols; ++c)
                for (int r = tid; r < rend; r += LU_THREADS) ab_put(a, j0 + r, c0 + c, Xc[r + c * ldx]);
        }
        lds_barrier();
    }

    if (wg == 0 && nb1 > 0) {
        // panel b+1 lives in Xc rows nbp .. ; rows beyond those the update touched come from the band
        const int R1 = (int)min((int64_t)(nb1 + a.kl), a.n - j1);
        const int have = (b >= 0) ? (int)min((int64_t)(nbp + a.kl), a.n - j0) - nbp : 0;
        cplx* P = Xc + nbp;
        load_tile(a, P, ldx, j1, j1, R1, nb1, have);
        lds_barrier();
        factor_panel(a, P, ldx, j1, nb1, R1, a.lt[(b + 1) & 1], red_v, red_i, piv_s);
    }
}

int lu_panel_width(int kl) {
    // one buffer of (nb + kl) rows and one of (2 nb + kl) rows, nb columns, padded, must fit in LDS
    const size_t lds = 160 * 1024 - 8 * 1024;
    for (int nb = 16; nb >= 4; nb /= 2) {
        size_t need = ((size_t)lds_ld(nb + kl) + (size_t)lds_ld(2 * nb + kl)) * nb * sizeof(cplx);
        if (need <= lds) return nb;
    }
    return 0;
}

simm_status band_lu(int64_t n, int kl, int ku, cplx* AB, int* ipiv, cplx* lt_scratch, int* info,
                    hipStream_t st) {
    const int nb = lu_panel_width(kl);
    if (nb == 0) {
        set_error("lower bandwidth too large for the LU kernel");
        return SIMM_EUNSUPPORTED;
    }
    LuArgs a;
    a.n = n;
    a.kl = kl;
    a.ku = ku;
    a.kv = kl + ku;
    a.ldab = 2 * kl + ku + 1;
    a.nb = nb;
    a.cw = nb;
    a.AB = AB;
    a.ipiv = ipiv;
    a.lt[0] = lt_scratch;
    a.lt[1] = lt_scratch + (size_t)(nb + kl) * nb;
    a.info = info;
    a.zidx = (int64_t)a.ldab * n;
    const size_t lds = ((size_t)lds_ld(nb + kl) * nb + (size_t)lds_ld(2 * nb + kl) * nb) * sizeof(cplx);
    const int grid = 2 + (a.kv + a.cw - 1) / a.cw;
    const int64_t nblk = (n + nb - 1) / nb;
    for (int64_t b = -1; b < nblk; ++b) {
        hipLaunchKernelGGL(k_band_lu_step, dim3(b < 0 ? 1 : grid), dim3(LU_THREADS), lds, st, a, b);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

size_t band_lu_scratch_elems(int kl) {
    const int nb = lu_panel_width(kl);
    return 2 * (size_t)(nb + kl) * (size_t)(nb > 0 ? nb : 1);
}

simm_status assemble_shifted(int64_t n, int kl, int ku, const cplx* A, int kla, int kua, const cplx* B, int klb,
                             int kub, cplx sigma, cplx* AB, hipStream_t st) {
    hipLaunchKernelGGL(k_assemble_shifted, dim3((unsigned)n), dim3(256), 0, st, n, kl, ku, A, kla, kua, B, klb, kub,
                       sigma, AB);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
