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
// Blocked right-looking schedule, one launch per panel of NB = 16 columns:
//   launch b:  every workgroup takes 16 of the columns right of panel b and
//              applies panel b's interchanges, the unit-lower triangular solve and
//              the rank-16 update (trailing window = rows of the panel + kl), and
//              workgroup 0, which owns panel b+1, then factors panel b+1.
// Each thread keeps one row of its window in registers; rows meet only through
// LDS at workgroup barriers.  Consecutive launches on one stream order the panels;
// no workgroup ever waits on another.
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

// a1: C = A - sigma B written into LU band storage (fill rows zeroed), formed in FP64
// and stored in the factor's precision.
template <typename CT>
__global__ void k_assemble_shifted(int64_t n, int kl, int ku, const cplx* __restrict__ A, int kla, int kua,
                                   const cplx* __restrict__ B, int klb, int kub, cplx sigma,
                                   CT* __restrict__ AB) {
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
        AB[(int64_t)r + c * ldab] = narrow<CT>(v);
    }
}

namespace {

constexpr int NB = 16;        // panel width
constexpr int SROW = NB + 1;  // LDS row stride (complex): 16 lanes writing 16-byte rows hit 16 bank groups
constexpr int CSTRIDE = NB + 2;   // candidate record: row (NB entries), reciprocal pivot, (max, position)

template <typename C>
struct LuArgs {
    int64_t n;
    int kl, ku, kv, ldab;
    C* AB;
    int* ipiv;       // 0-based global row of the pivot of each column
    C* LP;           // permuted multipliers of every panel: panel p at LP + p NB (NB+kl), column-major (NB+kl) x NB
    int* info;       // first singular column + 1 (INT_MAX if none)
    int64_t zidx;    // index of the zero entry stored after the band
    int64_t bs;      // > 0: block-diagonal mode, diagonal blocks of bs columns (workgroup row y: block y)
    int64_t row0;    // first row of the block (pivots and info are stored as global rows)
};

// Index of band entry (i, c), or of the zero entry when (i, c) lies outside the
// band: loads through it are unconditional, so all of a thread's loads are in flight together.
template <typename C>
__device__ inline int64_t ab_idx(const LuArgs<C>& a, int64_t i, int64_t c) {
    const int64_t d = i - c;
    const bool in = i >= 0 && i < a.n && c >= 0 && c < a.n && d >= -a.kv && d <= a.kl;
    return in ? (int64_t)(a.kv + d) + c * a.ldab : a.zidx;
}
template <typename C>
__device__ inline void ab_put(const LuArgs<C>& a, int64_t i, int64_t c, C v) {
    const int64_t d = i - c;
    if (i < 0 || i >= a.n || c < 0 || c >= a.n || d < -a.kv || d > a.kl) return;
    a.AB[(int64_t)(a.kv + d) + c * a.ldab] = v;
}

// Position that row i of the window held before the interchanges (t, pv[t]),
// t = 0 .. NB-1, were applied in order.
__device__ inline int trace_src(int i, const int* pv) {
    int pos = i;
#pragma unroll
    for (int t = NB - 1; t >= 0; --t) {
        const int p = pv[t];
        pos = (pos == t) ? p : ((pos == p) ? t : pos);
    }
    return pos;
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float dpp_d(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}

__device__ inline double rdlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ inline float rdlane_d(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }

// Maximum over the wavefront, returned to every lane: DPP within 16-lane rows
// (quad xor 1, quad xor 2, half-row mirror, row mirror), then row broadcasts of
// lanes 15 and 31 carry the row maxima to lane 63.
template <typename R>
__device__ inline R wave_max(R v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    v = fmax(v, dpp_d<0x140>(v));
    v = fmax(v, dpp_d<0x142, 0xA>(v));
    v = fmax(v, dpp_d<0x143, 0xC>(v));
    return rdlane_d(v, 63);
}

// Minimum over the wavefront (same DPP pattern as wave_max), returned to every lane.
__device__ inline int wave_min_int(int k) {
    k = min(k, __builtin_amdgcn_update_dpp(k, k, 0xB1, 0xf, 0xf, false));
    k = min(k, __builtin_amdgcn_update_dpp(k, k, 0x4E, 0xf, 0xf, false));
    k = min(k, __builtin_amdgcn_update_dpp(k, k, 0x141, 0xf, 0xf, false));
    k = min(k, __builtin_amdgcn_update_dpp(k, k, 0x140, 0xf, 0xf, false));
    k = min(k, __builtin_amdgcn_update_dpp(k, k, 0x142, 0xa, 0xf, false));
    k = min(k, __builtin_amdgcn_update_dpp(k, k, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(k, 63);
}

__device__ inline cplx rdlane(cplx v, int l) { return cplx{rdlane_d(v.re, l), rdlane_d(v.im, l)}; }
__device__ inline cplxf rdlane(cplxf v, int l) { return cplxf{rdlane_d(v.re, l), rdlane_d(v.im, l)}; }
// value of the partner lane (lane xor 1)
__device__ inline cplx swap_pair(cplx v) { return cplx{dpp_d<0xB1>(v.re), dpp_d<0xB1>(v.im)}; }
__device__ inline cplxf swap_pair(cplxf v) { return cplxf{dpp_d<0xB1>(v.re), dpp_d<0xB1>(v.im)}; }

// 1 / u by Smith's scaling (no overflow for any finite nonzero u), without branches.
__device__ inline cplx crecip(cplx u) {
    const bool big = fabs(u.re) >= fabs(u.im);
    const double p = big ? u.re : u.im, q = big ? u.im : u.re;
    const double s = q / p, d = 1.0 / (p + q * s);
    return big ? cplx{d, -s * d} : cplx{s * d, -d};
}
__device__ inline cplxf crecip(cplxf u) {
    const bool big = fabsf(u.re) >= fabsf(u.im);
    const float p = big ? u.re : u.im, q = big ? u.im : u.re;
    const float s = q / p, d = 1.0f / (p + q * s);
    return big ? cplxf{d, -s * d} : cplxf{s * d, -d};
}

// 16-byte (FP64) or 8-byte (FP32) LDS accesses of whole complex entries; every LDS
// buffer below is aligned to its entry size.
__device__ inline cplx ldsr(const cplx* p) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    return cplx{v.x, v.y};
}
__device__ inline void ldsw(cplx* p, cplx v) { *reinterpret_cast<double2*>(p) = double2{v.re, v.im}; }
__device__ inline cplxf ldsr(const cplxf* p) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    return cplxf{v.x, v.y};
}
__device__ inline void ldsw(cplxf* p, cplxf v) { *reinterpret_cast<float2*>(p) = float2{v.re, v.im}; }

template <typename C>
struct Real;
template <>
struct Real<cplx> {
    using T = double;
};
template <>
struct Real<cplxf> {
    using T = float;
};

// LDS layout of one step launch (complex entries of type C).
template <int T, typename C>
struct LuSmem {
    static constexpr int S = 0;                          // T x SROW   : window rows before interchanges
    static constexpr int LSH = S + T * SROW;             // NB x SROW  : diagonal block of the panel multipliers
    static constexpr int USH = LSH + NB * SROW;          // NB x SROW  : U12 block after the triangular solve
    static constexpr int CAND = USH + NB * SROW;         // 2 x (T/64) x CSTRIDE : each wave's pivot candidate
    static constexpr int END = CAND + 2 * (T / 64) * CSTRIDE;
    static constexpr size_t bytes = (size_t)END * sizeof(C) + NB * sizeof(int);
};

}  // namespace

namespace {

template <typename C>
struct FactorCtx {
    bool prow;       // this thread holds a row of the panel
    int nb1;         // panel width
    int64_t j1;      // first column (and row) of the panel
    int lane, wave;
    C* cand;         // 2 x waves x CSTRIDE
};

// Column step t of the panel factorization: partial pivoting by the largest
// |re| + |im| with the first position on ties (LAPACK's izamax rule).  Rows never
// move between threads: each thread carries the position `pos` its row holds, and
// an interchange just swaps two positions.  Per step one or two LDS barriers: the lane that
// holds each wave's candidate (the wave's largest entry, first position on ties)
// writes the (max, position) pair to the wave's record; after a barrier every lane
// reads the records, picks the winner, the winning lane writes its row and
// reciprocal pivot, and after a second barrier every lane reads that row with
// broadcast LDS reads (no lane reads on the chain).  A single-lane LDS write costs a
// full LDS pass for the CU, so only one wavefront writes a row.  With one
// wavefront the row goes with the pair, before a single barrier.
template <int T, int t, typename C>
__device__ __forceinline__ void factor_steps(const LuArgs<C>& a, C (&X)[NB], int& pos, const FactorCtx<C>& f) {
    using R = typename Real<C>::T;
    constexpr int W = T / 64;
    if (t < f.nb1) {
        const int buf = t & 1;
        const int64_t j = f.j1 + t;
        const int km = (int)min((int64_t)a.kl, a.n - 1 - j);
        const bool valid = f.prow && pos >= t && pos <= t + km;
        const R v = valid ? cabs1(X[t]) : R(-1);
        C inv_own = crecip(X[t]);                     // only the pivot's is used; computed by every
        asm volatile("" : "+v"(inv_own.re), "+v"(inv_own.im));   // lane here so it overlaps the reduction
        const R m = wave_max(v);
        const int key = (v == m) ? pos : 0x7fffffff;
        const int kmin = wave_min_int(key);
        const unsigned long long bal = __ballot(key == kmin);
        const int wl = bal ? __ffsll((long long)bal) - 1 : 0;
        if constexpr (W == 1) {
            if (f.lane == wl) {
                C* rec = f.cand + buf * CSTRIDE;
#pragma unroll
                for (int c = t; c < NB; ++c) ldsw(rec + c, X[c]);
                ldsw(rec + NB, inv_own);
                ldsw(rec + NB + 1, C{m, (R)kmin});
            }
        } else {
            // several wavefronts share the LDS: first only the (max, position) pairs
            if (f.lane == wl) ldsw(f.cand + (buf * W + f.wave) * CSTRIDE + NB + 1, C{m, (R)kmin});
        }
        lds_barrier();
        const C r0 = ldsr(f.cand + (buf * W) * CSTRIDE + NB + 1);
        R best = r0.re;
        int bpos = (int)r0.im, bw = 0;
#pragma unroll
        for (int w = 1; w < W; ++w) {
            const C rw = ldsr(f.cand + (buf * W + w) * CSTRIDE + NB + 1);
            const R vw = rw.re;
            const int pw = (int)rw.im;
            const bool take = vw > best || (vw == best && pw < bpos);
            best = take ? vw : best;
            bpos = take ? pw : bpos;
            bw = take ? w : bw;
        }
        const bool zero = !(best > R(0));
        if (zero) bpos = t;
        if (threadIdx.x == 0) {
            a.ipiv[j] = (int)(f.j1 + bpos + a.row0);
            // singular column: recorded; no interchange, no elimination
            if (zero) atomicMin(a.info, (int)(j + 1 + a.row0));
        }
        if constexpr (W > 1) {
            // then the winning wavefront's candidate lane publishes its row
            if (f.wave == bw && f.lane == wl) {
                C* rec = f.cand + (buf * W + bw) * CSTRIDE;
#pragma unroll
                for (int c = t; c < NB; ++c) ldsw(rec + c, X[c]);
                ldsw(rec + NB, inv_own);
            }
            lds_barrier();
        }
        if (!zero) {
            const C* win = f.cand + (buf * W + bw) * CSTRIDE;
            C u[NB + 1];
#pragma unroll
            for (int c = t; c <= NB; ++c) u[c] = ldsr(win + c);
            const int p0 = pos;
            pos = (p0 == t) ? bpos : ((p0 == bpos) ? t : p0);
            if (f.prow && pos > t) {
                const C l = X[t] * u[NB];
                X[t] = l;
#pragma unroll
                for (int c = t + 1; c < NB; ++c) X[c] = fms(X[c], l, u[c]);
            }
        }
        // column t's multipliers go to the band as computed now (later interchanges do not move them)
        if (f.prow && pos > t && pos - t <= a.kl) a.AB[(int64_t)(a.kv + pos - t) + j * a.ldab] = X[t];
    }
    if constexpr (t + 1 < NB) factor_steps<T, t + 1, C>(a, X, pos, f);
}

// v[ws] for a lane's ROWS (1 or 2) slots, without indexing the array by a variable
template <int ROWS, typename C>
__device__ __forceinline__ C pick_slot(const C (&v)[ROWS], int ws) {
    static_assert(ROWS == 1 || ROWS == 2, "one or two rows per lane");
    if constexpr (ROWS == 1) return v[0];
    else return csel(ws == 1, v[1], v[0]);
}

// The 16 column steps of a panel held by one wavefront, ROWS rows per lane (slot k of a
// lane: a panel row whose current position is pos[k]).  Pivot choice, interchanges (of
// positions), eliminations and the multipliers stored as computed are those of
// factor_steps; the pivot row and its reciprocal reach the other lanes by lane reads, so
// a column step needs no LDS and no barrier.
template <int ROWS, typename C, int t>
__device__ __forceinline__ void factor_wave_step(const LuArgs<C>& a, C (&X)[ROWS][NB], int (&pos)[ROWS],
                                                 const bool (&prow)[ROWS], int nb1, int64_t j1) {
    using R = typename Real<C>::T;
    if (t < nb1) {
        const int64_t j = j1 + t;
        const int km = (int)min((int64_t)a.kl, a.n - 1 - j);
        // this lane's candidate: the largest |re| + |im| of its valid rows, first position on ties
        R lv = R(-1);
        int lp = 0x7fffffff, ls = 0;
        C inv[ROWS];
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const bool valid = prow[k] && pos[k] >= t && pos[k] <= t + km;
            const R v = valid ? cabs1(X[k][t]) : R(-1);
            inv[k] = crecip(X[k][t]);   // only the pivot's is used; formed here beside the reduction
            asm volatile("" : "+v"(inv[k].re), "+v"(inv[k].im));
            const bool take = valid && (v > lv || (v == lv && pos[k] < lp));
            lv = take ? v : lv;
            lp = take ? pos[k] : lp;
            ls = take ? k : ls;
        }
        const R m = wave_max(lv);
        const int key = (lv == m) ? lp : 0x7fffffff;
        const int kmin = wave_min_int(key);
        const unsigned long long bal = __ballot(key == kmin);
        const int wl = bal ? __ffsll((long long)bal) - 1 : 0;
        const int ws = __builtin_amdgcn_readlane(ls, wl);
        const bool zero = !(m > R(0));
        const int bpos = zero ? t : kmin;
        if (threadIdx.x == 0) {
            a.ipiv[j] = (int)(j1 + bpos + a.row0);
            // singular column: recorded; no interchange, no elimination
            if (zero) atomicMin(a.info, (int)(j + 1 + a.row0));
        }
        if (!zero) {
            // the winning row, column by column, from the winning lane (its slot ws)
            C invs[ROWS], xt[ROWS];
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                invs[k] = inv[k];
                xt[k] = X[k][t];
            }
            const C uinv = rdlane(pick_slot<ROWS>(invs, ws), wl);
            C l[ROWS];
            bool el[ROWS];
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                const int p0 = pos[k];
                pos[k] = (p0 == t) ? bpos : ((p0 == bpos) ? t : p0);
                el[k] = prow[k] && pos[k] > t;
                l[k] = xt[k] * uinv;
                if (el[k]) X[k][t] = l[k];
            }
#pragma unroll
            for (int c = t + 1; c < NB; ++c) {
                C xc[ROWS];
#pragma unroll
                for (int k = 0; k < ROWS; ++k) xc[k] = X[k][c];
                const C uc = rdlane(pick_slot<ROWS>(xc, ws), wl);
#pragma unroll
                for (int k = 0; k < ROWS; ++k)
                    if (el[k]) X[k][c] = fms(X[k][c], l[k], uc);
            }
        }
        // column t's multipliers go to the band as computed now
#pragma unroll
        for (int k = 0; k < ROWS; ++k)
            if (prow[k] && pos[k] > t && pos[k] - t <= a.kl)
                a.AB[(int64_t)(a.kv + pos[k] - t) + j * a.ldab] = X[k][t];
    }
    if constexpr (t + 1 < NB) factor_wave_step<ROWS, C, t + 1>(a, X, pos, prow, nb1, j1);
}

template <int ROWS, typename C>
__device__ __forceinline__ void factor_wave(const LuArgs<C>& a, C (&X)[ROWS][NB], int (&pos)[ROWS],
                                            const bool (&prow)[ROWS], int nb1, int64_t j1) {
    factor_wave_step<ROWS, C, 0>(a, X, pos, prow, nb1, j1);
}

// U rows and permuted multipliers of a factored panel b+1 from one row (position pr).
template <typename C>
__device__ __forceinline__ void store_panel_row(const LuArgs<C>& a, const C (&X)[NB], int pr, bool prow, int nb1,
                                                int64_t j1, int64_t b) {
    // rows of U (final since their own step) to the band
    if (prow && pr < nb1) {
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (q >= pr && q < nb1 && q - pr <= a.kv) a.AB[(int64_t)(a.kv + pr - q) + (j1 + q) * a.ldab] = X[q];
    }
    // permuted multipliers of panel b+1 (entries left of the diagonal; zeros elsewhere
    // and in the rows past the matrix) for the next launch's update and the sweeps
    if (pr >= 0 && pr < NB + a.kl) {
        C* lp_out = a.LP + (b + 1) * (int64_t)(NB + a.kl) * NB + pr;
#pragma unroll
        for (int q = 0; q < NB; ++q)
            lp_out[(int64_t)q * (NB + a.kl)] = (prow && q < pr && q < nb1) ? X[q] : C{0, 0};
    }
}

}  // namespace

// One launch per panel.  Thread tid holds row tid of the window (rows j0 .. of the
// matrix, j0 = first row of panel b) for the 16 columns of its workgroup in
// registers, plus its row of panel b's permuted multipliers.
//   all workgroups: apply panel b's interchanges, the unit lower triangular solve
//                   on the top rows and the rank-NB update to their 16 columns;
//   workgroup 0:    its columns are panel b+1, which it then factors with partial
//                   pivoting, one column step per LDS barrier.
template <int T, typename C>
__global__ __launch_bounds__(T) void k_band_lu_step(LuArgs<C> a, int64_t b) {
    if (a.bs > 0) {
        // block-diagonal mode: the diagonal block of this workgroup row, as a matrix of
        // its own stored in place (its columns of the band, its panels of LP)
        const int64_t r0 = (int64_t)blockIdx.y * a.bs;
        a.n = min(a.bs, a.n - r0);
        a.AB += r0 * a.ldab;
        a.zidx -= r0 * a.ldab;
        a.ipiv += r0;
        a.LP += (r0 / NB) * (int64_t)(NB + a.kl) * NB;
        a.row0 = r0;
        if (b * NB >= a.n) return;   // a shorter last block is done
    }
    extern __shared__ double2 smem_raw[];
    C* smem = reinterpret_cast<C*>(smem_raw);
    using L = LuSmem<T, C>;
    // a prvalue: with two lvalue operands a struct-valued ?: selects between addresses and
    // puts its operands (the row registers) in scratch memory
    const auto zero_c = []() { return C{0, 0}; };
    C* S = smem + L::S;
    C* Lsh = smem + L::LSH;
    C* Ush = smem + L::USH;
    C* cand = smem + L::CAND;
    int* piv_s = reinterpret_cast<int*>(smem + L::END);

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wg = blockIdx.x;
    const int nbp = (b >= 0) ? (int)min((int64_t)NB, a.n - b * NB) : 0;   // width of panel b
    const int64_t j1 = (b >= 0) ? b * NB + nbp : 0;                       // first column of panel b+1
    const int64_t j0 = j1 - nbp;                                          // first row of the window
    const int nb1 = (int)max((int64_t)0, min((int64_t)NB, a.n - j1));     // width of panel b+1

    int64_t c0, c1;
    if (wg == 0) {
        c0 = j1;
        c1 = j1 + nb1;
    } else {
        if (b < 0) return;
        const int64_t jmax = min(a.n - 1, j1 - 1 + (int64_t)a.kv);
        c0 = j1 + nb1 + (int64_t)(wg - 1) * NB;
        c1 = min(c0 + NB, jmax + 1);
        if (c0 > jmax) return;
    }
    const int ncols = (int)(c1 - c0);
    // Only panel b = last can be narrower than NB, and no column lies right of it: every
    // launch that gets past here with b >= 0 has nbp == NB.
    if (ncols <= 0) return;
    const int Rb = (int)min((int64_t)(nbp + a.kl), a.n - j0);             // rows panel b updates
    const int R1 = (wg == 0) ? (int)min((int64_t)(nb1 + a.kl), a.n - j1) : 0;  // rows of panel b+1
    const int Rw = (wg == 0) ? nbp + R1 : Rb;                             // rows this workgroup holds
    const int r = tid;

    // ---- all global loads of the launch, issued together
    C X[NB], Lr[NB];
    {
        const bool mine = r < Rw;
#pragma unroll
        for (int c = 0; c < NB; ++c) X[c] = a.AB[(mine && c < ncols) ? ab_idx(a, j0 + r, c0 + c) : a.zidx];
        const C* lp_in = a.LP + (b >= 0 ? b : 0) * (int64_t)(NB + a.kl) * NB;
        const bool hasl = b >= 0 && r < Rb;
#pragma unroll
        for (int q = 0; q < NB; ++q) Lr[q] = hasl ? lp_in[(int64_t)q * (NB + a.kl) + r] : zero_c();
        if (b >= 0 && tid < NB) piv_s[tid] = (int)(a.ipiv[j0 + tid] - j0 - a.row0);
    }

    if (b >= 0) {
        // ---- interchanges of panel b: rows that move go through LDS
        if (r < Rb) {
#pragma unroll
            for (int c = 0; c < NB; ++c) ldsw(S + r * SROW + c, X[c]);
        }
        if (r < NB) {
#pragma unroll
            for (int q = 0; q < NB; ++q) ldsw(Lsh + r * SROW + q, Lr[q]);
        }
        lds_barrier();
        int pv[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) pv[t] = piv_s[t];
        if (r >= NB && r < Rb) {
            const int sr = trace_src(r, pv);
            if (sr != r) {
#pragma unroll
                for (int c = 0; c < NB; ++c) X[c] = ldsr(S + sr * SROW + c);
            }
        }
        // ---- unit lower triangular solve of the top NB rows (U12 = L11^{-1} A12), one
        // entry (i, c) of the NB x NB block per thread and round (E rounds): at step t
        // row t is final and goes to LDS, the rows below subtract L(i, t) times it.
        // Each entry sees the operations of a column-by-column forward substitution, in
        // the same order.
        {
            constexpr int E = (NB * NB + T - 1) / T;
            C xt[E];
            int ti[E], tc[E];
            bool tin[E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int e = tid + k * T;
                tin[k] = e < NB * NB;
                ti[k] = e / NB;
                tc[k] = e % NB;
                xt[k] = tin[k] ? ldsr(S + trace_src(ti[k], pv) * SROW + tc[k]) : zero_c();
            }
#pragma unroll
            for (int t = 0; t < NB; ++t) {
#pragma unroll
                for (int k = 0; k < E; ++k)
                    if (tin[k] && ti[k] == t) ldsw(Ush + t * SROW + tc[k], xt[k]);
                lds_barrier();
#pragma unroll
                for (int k = 0; k < E; ++k)
                    if (tin[k] && ti[k] > t)
                        xt[k] = fms(xt[k], ldsr(Lsh + ti[k] * SROW + t), ldsr(Ush + t * SROW + tc[k]));
            }
#pragma unroll
            for (int k = 0; k < E; ++k)
                if (tin[k] && tc[k] < ncols) ab_put(a, j0 + ti[k], c0 + tc[k], xt[k]);
        }
        lds_barrier();
        // ---- rank-NB update of rows NB .. Rb-1
        if constexpr (T == 256) {
            // lanes 2k and 2k+1 (rows r, r+1) share the update: the even lane takes
            // columns 0..7 of both rows, the odd lane columns 8..15, so that each LDS
            // read of U12 serves two rows (half the LDS traffic of one row per lane);
            // halves go to the partner lane and back with a lane swap.  Every entry gets
            // the same operations in the same order; rows outside NB .. Rb-1 pass through
            // with zero multipliers (rows above NB are not used after the solve).
            const bool odd = (tid & 1) != 0;
            constexpr int H = NB / 2;
            C A[H], B[H];
#pragma unroll
            for (int i = 0; i < H; ++i) {
                A[i] = csel(odd, X[H + i], X[i]);
                B[i] = swap_pair(csel(odd, X[i], X[H + i]));
            }
            const int cb = odd ? H : 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const C lq = swap_pair(Lr[q]);
#pragma unroll
                for (int i = 0; i < H; ++i) {
                    const C u = ldsr(Ush + q * SROW + cb + i);
                    A[i] = fms(A[i], Lr[q], u);
                    B[i] = fms(B[i], lq, u);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int i = 0; i < H; ++i) {
                const C back = swap_pair(B[i]);
                X[i] = csel(odd, back, A[i]);
                X[H + i] = csel(odd, A[i], back);
            }
            if (r >= NB && r < Rb && wg != 0) {
#pragma unroll
                for (int c = 0; c < NB; ++c)
                    if (c < ncols) ab_put(a, j0 + r, c0 + c, X[c]);
            }
        } else {
            if (r >= NB && r < Rb) {
#pragma unroll
                for (int q = 0; q < NB; ++q) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) X[c] = fms(X[c], Lr[q], ldsr(Ush + q * SROW + c));
                    __builtin_amdgcn_sched_barrier(0);
                }
                if (wg != 0) {
#pragma unroll
                    for (int c = 0; c < NB; ++c)
                        if (c < ncols) ab_put(a, j0 + r, c0 + c, X[c]);
                }
            }
        }
    }
    if (wg != 0) return;

    // ---- workgroup 0: factor panel b+1 (window rows nbp .., panel position pos = r - nbp at the start)
    if constexpr (T == 64) {
        // one wavefront holds the panel's rows, one per lane
        C Xs[1][NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) Xs[0][c] = X[c];
        int ps[1] = {r - nbp};
        const bool pw[1] = {ps[0] >= 0 && ps[0] < R1};
        factor_wave<1, C>(a, Xs, ps, pw, nb1, j1);
        store_panel_row(a, Xs[0], ps[0], pw[0], nb1, j1, b);
    } else if constexpr (T == 128) {
        // the panel's rows (at most NB + kl <= 112) go to wavefront 0, two per lane
        const int p = r - nbp;
        lds_barrier();
        if (p >= 0 && p < R1) {
#pragma unroll
            for (int c = 0; c < NB; ++c) ldsw(S + p * SROW + c, X[c]);
        }
        lds_barrier();
        if (wave != 0) return;
        C Xs[2][NB];
        int ps[2];
        bool pw[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = lane + 64 * k;
            ps[k] = i;
            pw[k] = i < R1;
#pragma unroll
            for (int c = 0; c < NB; ++c) Xs[k][c] = pw[k] ? ldsr(S + i * SROW + c) : zero_c();
        }
        factor_wave<2, C>(a, Xs, ps, pw, nb1, j1);
#pragma unroll
        for (int k = 0; k < 2; ++k) store_panel_row(a, Xs[k], ps[k], pw[k], nb1, j1, b);
    } else {
        FactorCtx<C> f;
        int pos = r - nbp;
        f.prow = pos >= 0 && pos < R1;
        f.nb1 = nb1;
        f.j1 = j1;
        f.lane = lane;
        f.wave = wave;
        f.cand = cand;
        factor_steps<T, 0, C>(a, X, pos, f);
        store_panel_row(a, X, pos, f.prow, nb1, j1, b);
    }
}

namespace {
template <int T, typename C>
simm_status launch_lu(const LuArgs<C>& a, hipStream_t st, const std::atomic<bool>* cancel, int64_t& launches) {
    const int grid = 2 + (a.kv + NB - 1) / NB;
    const int64_t len = a.bs > 0 ? std::min(a.bs, a.n) : a.n;               // columns of the longest block
    const unsigned gy = a.bs > 0 ? (unsigned)((a.n + a.bs - 1) / a.bs) : 1u;   // diagonal blocks
    const int64_t nblk = (len + NB - 1) / NB;
    const size_t lds = LuSmem<T, C>::bytes;
    if (!cancel) {
        for (int64_t b = -1; b < nblk; ++b)
            hipLaunchKernelGGL((k_band_lu_step<T, C>), dim3(b < 0 ? 1 : grid, gy), dim3(T), lds, st, a, b);
        launches = nblk + 1;
        return SIMM_OK;
    }
    // at most RING * BATCH launches queued ahead of the device, so that a cancel
    // takes effect within that many steps
    constexpr int BATCH = 64, RING = 4;
    hipEvent_t ev[RING] = {};
    for (auto& e : ev) SIMM_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    struct Release {
        hipEvent_t* e;
        ~Release() {
            for (int i = 0; i < RING; ++i) (void)hipEventDestroy(e[i]);
        }
    } release{ev};
    int64_t batch = 0;
    for (int64_t b = -1; b < nblk; b += BATCH, ++batch) {
        if (cancel->load(std::memory_order_relaxed)) {
            set_error("factorisation cancelled");
            return SIMM_ECANCELED;
        }
        hipEvent_t& e = ev[batch % RING];
        if (batch >= RING) SIMM_HIP_TRY(hipEventSynchronize(e));
        const int64_t bend = std::min<int64_t>(b + BATCH, nblk);
        for (int64_t q = b; q < bend; ++q)
            hipLaunchKernelGGL((k_band_lu_step<T, C>), dim3(q < 0 ? 1 : grid, gy), dim3(T), lds, st, a, q);
        launches += bend - b;
        SIMM_HIP_TRY(hipEventRecord(e, st));
    }
    return SIMM_OK;
}
}  // namespace

int lu_panel_width(int kl) {
    // the workgroup holds the 2 NB + kl rows of its window, one per thread, at most 512
    return (kl >= 0 && 2 * NB + kl <= 512) ? NB : 0;
}

namespace {
template <typename C>
simm_status band_lu_t(int64_t n, int kl, int ku, C* AB, int* ipiv, C* LP, int* info, int64_t bs, hipStream_t st,
                      const std::atomic<bool>* cancel, int64_t* launches) {
    if (bs < 0 || bs % NB != 0) {
        set_error("diagonal block length of the band LU must be a multiple of 16");
        return SIMM_EINVAL;
    }
    if (lu_panel_width(kl) == 0) {
        set_error("lower bandwidth too large for the LU kernel");
        return SIMM_EUNSUPPORTED;
    }
    LuArgs<C> a;
    a.n = n;
    a.kl = kl;
    a.ku = ku;
    a.kv = kl + ku;
    a.ldab = 2 * kl + ku + 1;
    a.AB = AB;
    a.ipiv = ipiv;
    a.LP = LP;
    a.info = info;
    a.zidx = (int64_t)a.ldab * n;
    a.bs = (bs > 0 && bs < n) ? bs : 0;
    a.row0 = 0;
    int64_t count = 0;
    // the smallest workgroup that holds the window: fewer wavefronts to meet at each
    // column step's barrier (the pivot and the arithmetic do not depend on the split)
    const int rows = 2 * NB + kl;
    const simm_status rc = (rows <= 64)    ? launch_lu<64, C>(a, st, cancel, count)
                           : (rows <= 128) ? launch_lu<128, C>(a, st, cancel, count)
                           : (rows <= 256) ? launch_lu<256, C>(a, st, cancel, count)
                                           : launch_lu<512, C>(a, st, cancel, count);
    if (launches) *launches = count;
    SIMM_TRY(rc);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}
}  // namespace

simm_status band_lu(int64_t n, int kl, int ku, cplx* AB, int* ipiv, cplx* LP, int* info, hipStream_t st,
                    const std::atomic<bool>* cancel, int64_t* launches, int64_t bs) {
    return band_lu_t(n, kl, ku, AB, ipiv, LP, info, bs, st, cancel, launches);
}

simm_status band_lu(int64_t n, int kl, int ku, cplxf* AB, int* ipiv, cplxf* LP, int* info, hipStream_t st,
                    const std::atomic<bool>* cancel, int64_t* launches, int64_t bs) {
    return band_lu_t(n, kl, ku, AB, ipiv, LP, info, bs, st, cancel, launches);
}

size_t band_lu_panel_elems(int64_t n, int kl) { return (size_t)((n + NB - 1) / NB) * (size_t)(NB + kl) * NB; }

simm_status assemble_shifted(int64_t n, int kl, int ku, const cplx* A, int kla, int kua, const cplx* B, int klb,
                             int kub, cplx sigma, cplx* AB, hipStream_t st) {
    hipLaunchKernelGGL(k_assemble_shifted<cplx>, dim3((unsigned)n), dim3(256), 0, st, n, kl, ku, A, kla, kua, B, klb,
                       kub, sigma, AB);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status assemble_shifted(int64_t n, int kl, int ku, const cplx* A, int kla, int kua, const cplx* B, int klb,
                             int kub, cplx sigma, cplxf* AB, hipStream_t st) {
    hipLaunchKernelGGL(k_assemble_shifted<cplxf>, dim3((unsigned)n), dim3(256), 0, st, n, kl, ku, A, kla, kua, B, klb,
                       kub, sigma, AB);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
