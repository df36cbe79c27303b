// Shifted Galerkin solves, quadrature sums, indicator norms and decisions for a
// batch of squares (Sec. 2 eqs. (many), (error), (y), (reduced); Sec. 3.1 eq.
// (DeltaSm), Definitions 3.1-3.2, Remark 3.3).
//
// One workgroup evaluates one (square, shift) pair.  The Schur factor T of H_m
// (packed upper triangle) sits in LDS; each wavefront takes a quadrature point at
// a time (four interleaved), lanes own rows of yhat, and the upper triangular system
// (I + (sigma - z) T) yhat = beta Q^H e_1 is solved by columns from the bottom,
// the new unknown formed by the lane that owns its row and broadcast with readlane.  With y = Q yhat:
//   e_m^T y = qlast . yhat  (residual, eq. (error)),  ||y|| = ||yhat||,
//   s = Q (sum_j w_j yhat_j) / (2 pi i),
// so the per-point work is one triangular solve.  Partial sums are combined across
// the wavefronts in a fixed order (bitwise reproducible).
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

constexpr int IND_THREADS = 256;
constexpr int IND_WAVES = IND_THREADS / 64;

__device__ inline double readlane_d(double v, int l) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ inline cplx readlane_c(cplx v, int l) { return mk(readlane_d(v.re, l), readlane_d(v.im, l)); }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ inline cplx wave_sum_c(cplx v) { return mk(wave_sum_d(v.re), wave_sum_d(v.im)); }

// Square geometry and quadrature node, in the operation order of the contour rule:
// corners counter-clockwise from centre + (w/2)(-1-i); edge a -> b carries
// z = a + (t+1)(b-a)/2 and weight omega (b-a)/2.
__device__ void node(double cx, double cy, double h, int e, double t, double om, cplx& z, cplx& wq) {
#pragma clang fp contract(off)
    const double sx[4] = {-1.0, 1.0, 1.0, -1.0};
    const double sy[4] = {-1.0, -1.0, 1.0, 1.0};
    const int e1 = (e + 1) & 3;
    const double ar = cx + sx[e] * h, ai = cy + sy[e] * h;
    const double br = cx + sx[e1] * h, bi = cy + sy[e1] * h;
    const double dr = br - ar, di = bi - ai;
    const double tp = t + 1.0;
    z = mk(ar + (tp * dr) / 2.0, ai + (tp * di) / 2.0);
    wq = mk((om * dr) / 2.0, (om * di) / 2.0);
}

}  // namespace

// LDS of one square's evaluation besides the Schur factor (dynamic LDS)
struct IndShared {
    cplx red[IND_WAVES][2][128];
    double redT[IND_WAVES], redR[IND_WAVES];
    cplx shat[2][128];
};

// One (square, shift) pair, by the whole workgroup; output slot `reg`.  Every operation
// and its order depend only on the square, the shift and the rule, so that the result
// does not depend on how the squares are dealt to workgroups.
__device__ __forceinline__ void eval_square(const ShiftDev& sh, int64_t level, int64_t ix, int64_t iy, int64_t reg,
                                            const IndicatorParams& prm, const RuleDev& rule, cplx* smem,
                                            IndShared& ls, double* indicator, double* rho_max, double* nsf_out,
                                            double* nsc_out, double* Tf_out, uint8_t* decision, cplx* sums,
                                            int m_sums) {
    auto& red = ls.red;
    auto& redT = ls.redT;
    auto& redR = ls.redR;
    auto& shat = ls.shat;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = sh.m;
    cplx* Ts = smem;
    const int nT = m * (m + 1) / 2;
    for (int e = threadIdx.x; e < nT; e += IND_THREADS) Ts[e] = sh.T[e];
    __syncthreads();

    // rows owned by this lane: i0 = lane, i1 = lane + 64
    const int i0 = lane, i1 = lane + 64;
    const cplx g0 = (i0 < m) ? sh.g[i0] : mk(0.0, 0.0);
    const cplx g1 = (i1 < m) ? sh.g[i1] : mk(0.0, 0.0);
    const cplx q0 = (i0 < m) ? sh.qlast[i0] : mk(0.0, 0.0);
    const cplx q1 = (i1 < m) ? sh.qlast[i1] : mk(0.0, 0.0);
    const cplx t00 = (i0 < m) ? Ts[i0 * (i0 + 1) / 2 + i0] : mk(0.0, 0.0);
    const cplx t11 = (i1 < m) ? Ts[i1 * (i1 + 1) / 2 + i1] : mk(0.0, 0.0);

    const double width = ldexp(prm.w1, (int)(1 - level));
    double cx, cy;
    {
#pragma clang fp contract(off)
        cx = prm.x0 + ((double)ix + 0.5) * width;
        cy = prm.y0 + ((double)iy + 0.5) * width;
    }
    const double h = width / 2.0;
    const int g = rule.g;
    const int npts = 12 * g;

    cplx sc0 = mk(0, 0), sc1 = mk(0, 0), sf0 = mk(0, 0), sf1 = mk(0, 0);
    double Tf = 0.0, rmax = 0.0;
    // Wave w takes the points q = w + 4 t in order of t, NP of them at a time: their
    // triangular solves share the LDS column reads and interleave NP independent chains
    // of lane broadcasts (per point, the operations and the accumulation order are those
    // of one point at a time).
    constexpr int NP = 4;
    const int npw = (npts - wave + IND_WAVES - 1) / IND_WAVES;
    const cplx one = mk(1.0, 0.0);
    for (int t0 = 0; t0 < npw; t0 += NP) {
        cplx alpha[NP], dinv0[NP], dinv1[NP], r0[NP], r1[NP], wq[NP];
        bool coarse[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int q = wave + IND_WAVES * min(t0 + u, npw - 1);   // past the end: a copy of the last point
            int e, idx;
            double t, om;
            if (q < 4 * g) {
                e = q / g;
                idx = q - e * g;
                t = rule.t1[idx];
                om = rule.w1[idx];
                coarse[u] = true;
            } else {
                const int q2 = q - 4 * g;
                e = q2 / (2 * g);
                idx = q2 - e * 2 * g;
                t = rule.t2[idx];
                om = rule.w2[idx];
                coarse[u] = false;
            }
            cplx z;
            node(cx, cy, h, e, t, om, z, wq[u]);
            alpha[u] = mk(sh.sig_re - z.re, sh.sig_im - z.im);
            dinv0[u] = cdiv(one, one + alpha[u] * t00);
            dinv1[u] = cdiv(one, one + alpha[u] * t11);
            r0[u] = g0;
            r1[u] = g1;
        }
        for (int j = m - 1; j >= 0; --j) {
            const int oj = j & 63;
            const cplx* col = Ts + j * (j + 1) / 2;
            cplx c0 = mk(0.0, 0.0), c1 = mk(0.0, 0.0);
            if (i0 < j) c0 = col[i0];
            if (i1 < j) c1 = col[i1];
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                // the lane owning row j forms y_j = r_j / (1 + alpha T_jj); one broadcast
                const cplx yj = (j < 64) ? readlane_c(r0[u] * dinv0[u], oj) : readlane_c(r1[u] * dinv1[u], oj);
                const cplx cj = alpha[u] * yj;
                if (i0 < j) r0[u] = fms(r0[u], c0, cj);
                if (i1 < j) r1[u] = fms(r1[u], c1, cj);
                if (i0 == j) r0[u] = yj;
                if (i1 == j) r1[u] = yj;
            }
        }
        // r0, r1 hold yhat of each point
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            if (t0 + u >= npw) break;
            const cplx dot = wave_sum_c(q0 * r0[u] + q1 * r1[u]);
            const double nrm2 = wave_sum_d(norm2(r0[u]) + norm2(r1[u]));
            const double rho = cabs(alpha[u]) * sh.h_last * cabs(dot) / sh.beta;
            rmax = fmax(rmax, rho);
            if (coarse[u]) {
                sc0 = fma_c(sc0, wq[u], r0[u]);
                sc1 = fma_c(sc1, wq[u], r1[u]);
            } else {
                sf0 = fma_c(sf0, wq[u], r0[u]);
                sf1 = fma_c(sf1, wq[u], r1[u]);
                Tf += cabs(wq[u]) * sqrt(nrm2);
            }
        }
    }
    red[wave][0][i0] = sc0;
    red[wave][0][i1] = sc1;
    red[wave][1][i0] = sf0;
    red[wave][1][i1] = sf1;
    if (lane == 0) {
        redT[wave] = Tf;
        redR[wave] = rmax;
    }
    __syncthreads();
    if (wave == 0) {
        cplx c0 = red[0][0][i0], c1 = red[0][0][i1], f0 = red[0][1][i0], f1 = red[0][1][i1];
        double T = redT[0], R = redR[0];
        for (int w = 1; w < IND_WAVES; ++w) {
            c0 = c0 + red[w][0][i0];
            c1 = c1 + red[w][0][i1];
            f0 = f0 + red[w][1][i0];
            f1 = f1 + red[w][1][i1];
            T += redT[w];
            R = fmax(R, redR[w]);
        }
        const double twopi = 6.283185307179586;
        const double nsc = sqrt(wave_sum_d(norm2(c0) + norm2(c1))) / twopi;
        const double nsf = sqrt(wave_sum_d(norm2(f0) + norm2(f1))) / twopi;
        const double Tfv = T / twopi;
        shat[0][i0] = c0;
        shat[0][i1] = c1;
        shat[1][i0] = f0;
        shat[1][i1] = f1;
        if (lane == 0) {
            const bool resolvable = R <= prm.eps0;
            const bool admissible = (nsf > prm.tau * Tfv) && (nsf > prm.delta0 * nsc);
            if (indicator) indicator[reg] = nsf / nsc;
            if (rho_max) rho_max[reg] = R;
            if (nsf_out) nsf_out[reg] = nsf;
            if (nsc_out) nsc_out[reg] = nsc;
            if (Tf_out) Tf_out[reg] = Tfv;
            if (decision) decision[reg] = (uint8_t)(!resolvable ? SIMM_UNRESOLVED : (admissible ? SIMM_ADMISSIBLE : SIMM_REJECTED));
        }
    }
    if (sums != nullptr) {
        __syncthreads();
        // s = Q shat / (2 pi i): waves 0/1 form s_c, waves 2/3 form s_f
        const int which = wave >> 1;
        const int i = (wave & 1) * 64 + lane;
        if (i < m_sums) {
            cplx acc = mk(0.0, 0.0);
            if (i < m) {
                for (int k = 0; k < m; ++k) acc = fma_c(acc, sh.Q[i + (int64_t)k * m], shat[which][k]);
            }
            const double twopi = 6.283185307179586;
            // x / (2 pi i) = (im, -re) / (2 pi)
            sums[((int64_t)reg * 2 + which) * m_sums + i] = mk(acc.im / twopi, -acc.re / twopi);
        }
    }
}

__global__ __launch_bounds__(IND_THREADS) void k_indicators(const ShiftDev* __restrict__ shifts,
                                                            const int64_t* __restrict__ regions, int64_t nreg,
                                                            IndicatorParams prm, RuleDev rule, double* indicator,
                                                            double* rho_max, double* nsf_out, double* nsc_out,
                                                            double* Tf_out, uint8_t* decision, cplx* sums,
                                                            int m_sums) {
    extern __shared__ cplx smem[];
    __shared__ IndShared ls;
    const int64_t reg = blockIdx.x;
    if (reg >= nreg) return;
    const ShiftDev sh = shifts[regions[4 * reg + 3]];
    eval_square(sh, regions[4 * reg + 0], regions[4 * reg + 1], regions[4 * reg + 2], reg, prm, rule, smem, ls,
                indicator, rho_max, nsf_out, nsc_out, Tf_out, decision, sums, m_sums);
}

// Persistent form over the squares of many pencils: rows of 5 int64 (level, ix, iy,
// shift, geometry), the row count read from device memory (so that one launch shape,
// e.g. inside a captured graph, serves every level), the square geometry and thresholds
// of each pencil in geo[].  Workgroup b takes rows b, b + gridDim.x, ...
__global__ __launch_bounds__(IND_THREADS) void k_indicators_persist(
    const ShiftDev* __restrict__ shifts, const int64_t* __restrict__ rows, const int64_t* __restrict__ nrows,
    const IndicatorParams* __restrict__ geo, RuleDev rule, double* indicator, double* rho_max, double* nsf_out,
    double* nsc_out, double* Tf_out, uint8_t* decision, cplx* sums, int m_sums) {
    extern __shared__ cplx smem[];
    __shared__ IndShared ls;
    const int64_t N = *nrows;
    for (int64_t reg = blockIdx.x; reg < N; reg += gridDim.x) {
        const int64_t* row = rows + 5 * reg;
        const ShiftDev sh = shifts[row[3]];
        const IndicatorParams prm = geo[row[4]];
        eval_square(sh, row[0], row[1], row[2], reg, prm, rule, smem, ls, indicator, rho_max, nsf_out, nsc_out,
                    Tf_out, decision, sums, m_sums);
        __syncthreads();   // LDS is reused by the next row
    }
}

// Fine-rule solutions of one square (the 2g-point rule of eq. (XLXf)): for each node
// z_j, y_j = Q yhat_j with (I + (sigma - z_j) T) yhat_j = beta Q^H e_1, the Galerkin
// solution of eq. (y) in the Arnoldi basis; row j of Y (stride ldy) holds y_j.  With
// conj_nodes the nodes are conjugated: the shift then belongs to the conjugate-transposed
// pencil at conj(sigma), whose resolvent at conj(z_j) is (A - z_j B)^{-H}.  cw, when
// given, receives c_j = w_j / (2 pi i).  Workgroup b's wave w takes point 4 b + w.
__global__ __launch_bounds__(IND_THREADS) void k_fine_solutions(ShiftDev sh, IndicatorParams prm, RuleDev rule,
                                                                int level, int64_t ix, int64_t iy, int conj_nodes,
                                                                cplx* __restrict__ Y, int ldy, cplx* __restrict__ cw,
                                                                double* __restrict__ rho) {
    extern __shared__ cplx smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = sh.m;
    cplx* Ts = smem;
    const int nT = m * (m + 1) / 2;
    for (int e = threadIdx.x; e < nT; e += IND_THREADS) Ts[e] = sh.T[e];
    __syncthreads();
    const int i0 = lane, i1 = lane + 64;
    const cplx g0 = (i0 < m) ? sh.g[i0] : mk(0.0, 0.0);
    const cplx g1 = (i1 < m) ? sh.g[i1] : mk(0.0, 0.0);
    const cplx t00 = (i0 < m) ? Ts[i0 * (i0 + 1) / 2 + i0] : mk(0.0, 0.0);
    const cplx t11 = (i1 < m) ? Ts[i1 * (i1 + 1) / 2 + i1] : mk(0.0, 0.0);
    const double width = ldexp(prm.w1, 1 - level);
    double cx, cy;
    {
#pragma clang fp contract(off)
        cx = prm.x0 + ((double)ix + 0.5) * width;
        cy = prm.y0 + ((double)iy + 0.5) * width;
    }
    const double h = width / 2.0;
    const int g2 = 2 * rule.g;
    const int nf = 4 * g2;
    const cplx one = mk(1.0, 0.0);
    const double twopi = 6.283185307179586;
    const int q = (int)blockIdx.x * IND_WAVES + wave;
    if (q < nf) {
        const int e = q / g2;
        const int idx = q - e * g2;
        cplx z, wq;
        node(cx, cy, h, e, rule.t2[idx], rule.w2[idx], z, wq);
        if (conj_nodes) z.im = -z.im;
        const cplx alpha = mk(sh.sig_re - z.re, sh.sig_im - z.im);
        const cplx dinv0 = cdiv(one, one + alpha * t00);
        const cplx dinv1 = cdiv(one, one + alpha * t11);
        cplx r0 = g0, r1 = g1;
        for (int j = m - 1; j >= 0; --j) {
            const int oj = j & 63;
            const cplx* col = Ts + j * (j + 1) / 2;
            const cplx yj = (j < 64) ? readlane_c(r0 * dinv0, oj) : readlane_c(r1 * dinv1, oj);
            const cplx cj = alpha * yj;
            if (i0 < j) r0 = fms(r0, col[i0], cj);
            if (i1 < j) r1 = fms(r1, col[i1], cj);
            if (i0 == j) r0 = yj;
            if (i1 == j) r1 = yj;
        }
        // y = Q yhat: the lanes keep their rows of y, yhat_k is broadcast
        cplx y0 = mk(0.0, 0.0), y1 = mk(0.0, 0.0);
        for (int k = 0; k < m; ++k) {
            const cplx yk = (k < 64) ? readlane_c(r0, k & 63) : readlane_c(r1, k & 63);
            if (i0 < m) y0 = fma_c(y0, sh.Q[i0 + (int64_t)k * m], yk);
            if (i1 < m) y1 = fma_c(y1, sh.Q[i1 + (int64_t)k * m], yk);
        }
        if (i0 < m) Y[(int64_t)q * ldy + i0] = y0;
        if (i1 < m) Y[(int64_t)q * ldy + i1] = y1;
        if (cw != nullptr && lane == 0) cw[q] = mk(wq.im / twopi, -wq.re / twopi);
        if (rho != nullptr) {
            // residual of this node's reduced solve, eq. (error): |sigma - z| h_{m+1,m} |e_m^T y| / beta
            const cplx ym = (m - 1 < 64) ? readlane_c(y0, (m - 1) & 63) : readlane_c(y1, (m - 1) & 63);
            if (lane == 0) rho[q] = cabs(alpha) * sh.h_last * cabs(ym) / sh.beta;
        }
    }
}

simm_status fine_solutions(const ShiftDev& sh, const IndicatorParams& prm, const RuleDev& rule, int level, int64_t ix,
                           int64_t iy, bool conj_nodes, cplx* Y, int ldy, cplx* cw, double* rho, hipStream_t st) {
    if (sh.m > 128 || ldy < sh.m) {
        set_error("fine_solutions: Krylov dimension above 128 or row stride below it");
        return SIMM_EUNSUPPORTED;
    }
    const size_t lds = sizeof(cplx) * (size_t)(sh.m * (sh.m + 1) / 2 + 1);
    const int nf = 8 * rule.g;
    hipLaunchKernelGGL(k_fine_solutions, dim3((unsigned)((nf + IND_WAVES - 1) / IND_WAVES)), dim3(IND_THREADS), lds,
                       st, sh, prm, rule, level, ix, iy, conj_nodes ? 1 : 0, Y, ldy, cw, rho);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status indicators_persist(const ShiftDev* shifts_dev, int mmax, const int64_t* rows, const int64_t* nrows,
                               const IndicatorParams* geo, const RuleDev& rule, int grid, double* indicator,
                               double* rho_max, double* nsf, double* nsc, double* Tf, uint8_t* decision, cplx* sums,
                               int m_sums, hipStream_t st) {
    if (mmax > 128 || (sums != nullptr && m_sums > 128)) {
        set_error("Krylov dimension above 128");
        return SIMM_EUNSUPPORTED;
    }
    const size_t lds = sizeof(cplx) * (size_t)(mmax * (mmax + 1) / 2 + 1);
    hipLaunchKernelGGL(k_indicators_persist, dim3((unsigned)grid), dim3(IND_THREADS), lds, st, shifts_dev, rows, nrows,
                       geo, rule, indicator, rho_max, nsf, nsc, Tf, decision, sums, m_sums);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

// Residuals of the reduced solves of whole cells straight from the Arnoldi matrix, for
// the association of the level-1 cells (which needs only whether a shift resolves a
// cell, Definition 3.1).  With M = I + (sigma - z) H_m upper Hessenberg and
// y = beta M^{-1} e_1, the cofactor of M's (1, m) entry is the product of M's
// subdiagonal, so e_m^T y = beta prod_{i<m} (sigma - z) h_{i+1,i} / det M and eq. (error)
// becomes
//     rho = |sigma - z|^m h_{m+1,m} prod_{i<m} h_{i+1,i} / |det M|.
// det M comes from Gaussian elimination with partial pivoting on M's rows, one row after
// another (a Hessenberg row meets only the current one), so a point needs O(m) storage:
// the current row over the wavefront's lanes (two entries a lane), H packed in LDS.
// Magnitudes are carried as (mantissa, exponent) pairs, so no product overflows.  Grid
// (cells, point groups); each workgroup raises the cell's maximum (non-negative doubles
// ordered as their bit patterns), so the result does not depend on the order.
namespace {
__device__ inline int hpk(int j) { return j * (j + 3) / 2; }   // packed column j: rows 0 .. min(j+1, m-1)
}  // namespace

__global__ __launch_bounds__(256) void k_cells_resid(const cplx* __restrict__ H, int ldh, int m, double hlast,
                                                     double sig_re, double sig_im, const int64_t* __restrict__ cells,
                                                     int level, IndicatorParams prm, RuleDev rule, int pts_per_wg,
                                                     unsigned long long* __restrict__ rbits) {
    extern __shared__ double2 hsm[];
    cplx* Hs = reinterpret_cast<cplx*>(hsm);
    double* sub = reinterpret_cast<double*>(Hs + hpk(m));   // [0]: sum of log h_{i+1,i}, i < m-1
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < m; ++j) {
        const int rows = min(j + 2, m);
        for (int i = threadIdx.x; i < rows; i += 256) Hs[hpk(j) + i] = H[i + (int64_t)j * ldh];
    }
    if (wave == 0) {
        double acc = 0.0;
        for (int i = lane; i < m - 1; i += 64) acc += log(cabs(H[(i + 1) + (int64_t)i * ldh]));
        acc = wave_sum_d(acc);
        if (lane == 0) sub[0] = acc;
    }
    __syncthreads();
    const double logsub = sub[0];
    const int64_t ix = cells[2 * blockIdx.x], iy = cells[2 * blockIdx.x + 1];
    const double width = ldexp(prm.w1, (int)(1 - level));
    double cx, cy;
    {
#pragma clang fp contract(off)
        cx = prm.x0 + ((double)ix + 0.5) * width;
        cy = prm.y0 + ((double)iy + 0.5) * width;
    }
    const double h = width / 2.0;
    const int g = rule.g;
    const int npts = 12 * g;
    const int q0 = blockIdx.y * pts_per_wg, q1 = min(npts, q0 + pts_per_wg);
    const int j0 = lane, j1 = lane + 64;
    const double ln2 = 0.6931471805599453;
    double rmax = 0.0;
    for (int q = q0 + wave; q < q1; q += 4) {
        int e, idx;
        double t, om;
        if (q < 4 * g) {
            e = q / g;
            idx = q - e * g;
            t = rule.t1[idx];
            om = rule.w1[idx];
        } else {
            const int q2 = q - 4 * g;
            e = q2 / (2 * g);
            idx = q2 - e * 2 * g;
            t = rule.t2[idx];
            om = rule.w2[idx];
        }
        cplx z, wq;
        node(cx, cy, h, e, t, om, z, wq);
        const cplx al = mk(sig_re - z.re, sig_im - z.im);
        // row 0 of M
        cplx r0 = (j0 < m) ? al * Hs[hpk(j0)] : mk(0.0, 0.0);
        cplx r1 = (j1 < m) ? al * Hs[hpk(j1)] : mk(0.0, 0.0);
        if (j0 == 0) r0 = r0 + mk(1.0, 0.0);
        double pm = 1.0;   // |det M| = pm 2^pe
        int pe = 0;
        bool singular = false;
        for (int k = 0; k + 1 < m; ++k) {
            // row k+1 of M on columns j >= k
            cplx n0 = mk(0.0, 0.0), n1 = mk(0.0, 0.0);
            if (j0 >= k && j0 < m) n0 = al * Hs[hpk(j0) + k + 1];
            if (j1 >= k && j1 < m) n1 = al * Hs[hpk(j1) + k + 1];
            if (j0 == k + 1) n0 = n0 + mk(1.0, 0.0);
            if (j1 == k + 1) n1 = n1 + mk(1.0, 0.0);
            const cplx rk = (k < 64) ? readlane_c(r0, k) : readlane_c(r1, k - 64);
            const cplx nk = al * Hs[hpk(k) + k + 1];
            const bool use_n = cabs1(nk) > cabs1(rk);
            const cplx pk = use_n ? nk : rk, ok = use_n ? rk : nk;
            const double mag = cabs(pk);
            if (!(mag > 0.0)) {
                singular = true;
                break;
            }
            int ex;
            pm = frexp(pm * mag, &ex);
            pe += ex;
            const cplx l = cdiv(ok, pk);
            const cplx p0 = use_n ? n0 : r0, o0 = use_n ? r0 : n0;
            const cplx p1 = use_n ? n1 : r1, o1 = use_n ? r1 : n1;
            r0 = fms(o0, l, p0);
            r1 = fms(o1, l, p1);
        }
        double rho;
        if (hlast == 0.0) {
            rho = 0.0;
        } else {
            const cplx last = ((m - 1) < 64) ? readlane_c(r0, m - 1) : readlane_c(r1, m - 65);
            const double ml = cabs(last);
            if (singular || !(ml > 0.0)) {
                rho = INFINITY;
            } else {
                int ex;
                pm = frexp(pm * ml, &ex);
                pe += ex;
                const double logdet = log(pm) + pe * ln2;
                rho = exp((double)m * log(cabs(al)) + log(hlast) + logsub - logdet);
                if (!(rho <= 1.7976931348623157e308)) rho = INFINITY;
            }
        }
        rmax = fmax(rmax, rho);
    }
#pragma unroll
    for (int msk = 32; msk >= 1; msk >>= 1) rmax = fmax(rmax, __shfl_xor(rmax, msk, 64));
    if (lane == 0) atomicMax(rbits + blockIdx.x, (unsigned long long)__double_as_longlong(rmax));
}

simm_status cells_resid(const cplx* H, int ldh, int m, double hlast, cplx sigma, const int64_t* cells, int64_t ncell,
                        int level, const IndicatorParams& prm, const RuleDev& rule, unsigned long long* rbits,
                        hipStream_t st) {
    if (ncell <= 0) return SIMM_OK;
    if (ncell > INT_MAX) {
        set_error("too many squares in one call");
        return SIMM_EINVAL;
    }
    if (m < 1 || m > 128) {
        set_error("Krylov dimension outside 1..128");
        return SIMM_EUNSUPPORTED;
    }
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, st, rbits, (int)ncell);
    constexpr int PTS = 16;   // points per workgroup: four per wavefront
    const int groups = (12 * rule.g + PTS - 1) / PTS;
    const size_t lds = sizeof(cplx) * (size_t)(m * (m + 3) / 2 + 2);
    hipLaunchKernelGGL(k_cells_resid, dim3((unsigned)ncell, (unsigned)groups), dim3(256), lds, st, H, ldh, m, hlast,
                       sigma.re, sigma.im, cells, level, prm, rule, PTS, rbits);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status indicators(const ShiftDev* shifts_dev, int mmax, const int64_t* regions, int64_t nreg,
                       const IndicatorParams& prm, const RuleDev& rule, double* indicator, double* rho_max,
                       double* nsf, double* nsc, double* Tf, uint8_t* decision, cplx* sums, int m_sums,
                       hipStream_t st) {
    if (nreg <= 0) return SIMM_OK;
    if (mmax > 128) {
        set_error("Krylov dimension above 128");
        return SIMM_EUNSUPPORTED;
    }
    if (sums != nullptr && m_sums > 128) {
        set_error("m_max above 128");
        return SIMM_EUNSUPPORTED;
    }
    const size_t lds = sizeof(cplx) * (size_t)(mmax * (mmax + 1) / 2 + 1);
    for (int64_t r0 = 0; r0 < nreg; r0 += 1 << 30) {
        const int64_t cnt = std::min<int64_t>(nreg - r0, (int64_t)1 << 30);
        hipLaunchKernelGGL(k_indicators, dim3((unsigned)cnt), dim3(IND_THREADS), lds, st, shifts_dev,
                           regions + 4 * r0, cnt, prm, rule, indicator ? indicator + r0 : nullptr,
                           rho_max ? rho_max + r0 : nullptr, nsf ? nsf + r0 : nullptr, nsc ? nsc + r0 : nullptr,
                           Tf ? Tf + r0 : nullptr, decision ? decision + r0 : nullptr,
                           sums ? sums + (size_t)r0 * 2 * m_sums : nullptr, m_sums);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
