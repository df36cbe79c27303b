// Schur form H_m = Q T Q^H of the Arnoldi Hessenberg matrix, once per shift.
//
// The shifted Galerkin systems (I + (sigma - z_j) H_m) y_j = beta e_1 of Sec. 2,
// eq. (many), become (I + (sigma - z_j) T) yhat_j = beta Q^H e_1 with y_j = Q yhat_j:
// an upper triangular solve per quadrature point.  Sec. 3.2 of the paper uses an
// eigendecomposition H_m = P D P^{-1} instead; the unitary Schur basis gives the same
// rational functions of z without inverting a possibly ill-conditioned P.  The
// diagonal of T holds the eigenvalues theta of H_m (Ritz values sigma + 1/theta).
//
// Method: complex single-shift QR iteration on the Hessenberg matrix (Wilkinson
// shift from the trailing 2x2 block, exceptional shifts after 10 and 20 stalled
// iterations, deflation when |h_{k,k-1}| <= eps (|h_{k-1,k-1}| + |h_{k,k}|)), bulge
// chased with Givens rotations applied to the whole matrix so that the full upper
// triangular T results.  One wavefront holds the Hessenberg matrix in LDS (packed by
// columns with room for the bulge) and records the rotations; a second kernel
// replays them on the rows of Q (rows are independent).
#include "common.hpp"
#include "kernels.hpp"

namespace simm {

namespace {

struct Rot {
    int k;
    int pad;
    double c;
    cplx s;
};

__device__ inline int hoff(int j) { return j * (j + 5) / 2; }   // column j holds rows 0 .. j+2

__device__ inline cplx csqrt_d(cplx z) {
    // principal square root
    const double r = hypot(z.re, z.im);
    if (r == 0.0) return mk(0.0, 0.0);
    double a = sqrt(0.5 * (r + fabs(z.re)));
    double b = z.im / (2.0 * a);
    if (z.re >= 0.0) return mk(a, b);
    return (z.im >= 0.0) ? mk(fabs(b), a) : mk(fabs(b), -a);
}

// Givens rotation G = [[c, s], [-conj(s), c]] (c real) with G [x; y] = [r; 0]
// (c = |x| / n, s = (x / |x|) conj(y) / n, r = (x / |x|) n, n = sqrt(|x|^2 + |y|^2);
// entries of H_m are far from the double range limits, so the squares are safe).
__device__ inline void givens(cplx x, cplx y, double& c, cplx& s, cplx& r) {
    const double ax2 = x.re * x.re + x.im * x.im, ay2 = y.re * y.re + y.im * y.im;
    if (ay2 == 0.0) {
        c = 1.0;
        s = mk(0.0, 0.0);
        r = x;
    } else if (ax2 == 0.0) {
        const double ay = sqrt(ay2);
        c = 0.0;
        s = mk(y.re / ay, -y.im / ay);
        r = mk(ay, 0.0);
    } else {
        const double ax = sqrt(ax2), nrm = sqrt(ax2 + ay2);
        const double inv_ax = 1.0 / ax, inv_n = 1.0 / nrm;
        c = ax * inv_n;
        const cplx ph = mk(x.re * inv_ax, x.im * inv_ax);
        s = mk((ph.re * y.re + ph.im * y.im) * inv_n, (ph.im * y.re - ph.re * y.im) * inv_n);   // ph conj(y) / n
        r = mk(ph.re * nrm, ph.im * nrm);
    }
}

constexpr int MAX_SCHUR_M = 128;

// The QR kernel is one wavefront: its LDS accesses execute in program order, so
// ordering them needs only a compiler barrier, not a workgroup barrier.
__device__ inline void wave_sync() { asm volatile("" ::: "memory"); }

}  // namespace

__global__ __launch_bounds__(64) void k_hess_qr(const cplx* __restrict__ Hin, int ldh, int m, Rot* rots, int max_rot,
                                                int* nrot_out, cplx* T_out, int* status) {
    extern __shared__ cplx Hs[];
    const int lane = threadIdx.x;
    auto H = [&](int i, int j) -> cplx& { return Hs[hoff(j) + i]; };
    // load the m x m Hessenberg part (rows 0 .. j+1 of column j; bulge slot zero)
    for (int j = 0; j < m; ++j)
        for (int i = lane; i <= j + 2; i += 64) Hs[hoff(j) + i] = (i <= j + 1 && i < m) ? Hin[i + (int64_t)j * ldh] : mk(0.0, 0.0);
    wave_sync();

    const double eps = 2.220446049250313e-16;
    int nrot = 0;
    int ihi = m - 1;
    int its = 0;
    int fail = 0;
    while (ihi > 0) {
        // deflation point: the largest k <= ihi with a negligible subdiagonal entry,
        // every lane testing its own k (k = lane + 1, lane + 65)
        int l = 0;
        {
            double dsum = -1.0;   // sum of |diag| over 0..ihi, only if some test needs it
            int kbest = 0;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = lane + 1 + 64 * u;
                bool small = false;
                double tst = 0.0;
                if (k <= ihi) {
                    tst = cabs1(H(k - 1, k - 1)) + cabs1(H(k, k));
                    small = tst != 0.0 && cabs1(H(k, k - 1)) <= eps * tst;
                }
                if (__ballot(k <= ihi && tst == 0.0)) {
                    if (dsum < 0.0) {
                        double acc = 0.0;
                        for (int i = lane; i <= ihi; i += 64) acc += cabs1(H(i, i));
#pragma unroll
                        for (int msk = 32; msk >= 1; msk >>= 1) acc += __shfl_xor(acc, msk, 64);
                        dsum = (acc == 0.0) ? 1.0 : acc;
                    }
                    if (k <= ihi && tst == 0.0) small = cabs1(H(k, k - 1)) <= eps * dsum;
                }
                if (small) kbest = max(kbest, k);
            }
#pragma unroll
            for (int msk = 32; msk >= 1; msk >>= 1) kbest = max(kbest, __shfl_xor(kbest, msk, 64));
            l = kbest;
        }
        if (l > 0) {
            if (lane == 0) H(l, l - 1) = mk(0.0, 0.0);
            wave_sync();
        }
        if (l >= ihi) {
            --ihi;
            its = 0;
            continue;
        }
        if (its >= 40) {
            fail = 1;
            break;
        }
        ++its;
        cplx mu;
        if (its == 10) {
            const cplx d = H(ihi, ihi);
            mu = mk(d.re + 0.75 * fabs(H(ihi, ihi - 1).re), d.im);
        } else if (its == 20) {
            const cplx d = H(l, l);
            mu = mk(d.re + 0.75 * fabs(H(l + 1, l).re), d.im);
        } else {
            const cplx a = H(ihi - 1, ihi - 1), b = H(ihi - 1, ihi), c = H(ihi, ihi - 1), d = H(ihi, ihi);
            const cplx half = mk(0.5 * (a.re - d.re), 0.5 * (a.im - d.im));
            const cplx disc = csqrt_d(half * half + b * c);
            const cplx tr2 = mk(0.5 * (a.re + d.re), 0.5 * (a.im + d.im));
            const cplx m1 = tr2 + disc, m2 = tr2 - disc;
            mu = (cabs(m1 - d) <= cabs(m2 - d)) ? m1 : m2;
        }
        for (int k = l; k < ihi; ++k) {
            cplx x, y;
            if (k == l) {
                x = H(l, l) - mu;
                y = H(l + 1, l);
            } else {
                x = H(k, k - 1);
                y = H(k + 1, k - 1);
            }
            double c;
            cplx s, r;
            givens(x, y, c, s, r);
            wave_sync();
            int jstart = k;
            if (k > l) {
                if (lane == 0) {
                    H(k, k - 1) = r;
                    H(k + 1, k - 1) = mk(0.0, 0.0);
                }
            } else {
                jstart = l;
            }
            // G from the left: rows k, k+1, columns jstart .. m-1
            for (int j = jstart + lane; j < m; j += 64) {
                const cplx hk = H(k, j), hk1 = H(k + 1, j);
                H(k, j) = mk(c * hk.re, c * hk.im) + s * hk1;
                H(k + 1, j) = mk(c * hk1.re, c * hk1.im) - conj(s) * hk;
            }
            wave_sync();
            // G^H from the right: columns k, k+1, rows 0 .. min(k+2, ihi)
            const int ilast = min(k + 2, ihi);
            for (int i = lane; i <= ilast; i += 64) {
                const cplx hik = H(i, k), hik1 = H(i, k + 1);
                H(i, k) = mk(c * hik.re, c * hik.im) + hik1 * conj(s);
                H(i, k + 1) = mk(c * hik1.re, c * hik1.im) - hik * s;
            }
            wave_sync();
            if (lane == 0) {
                if (nrot < max_rot) {
                    Rot rr;
                    rr.k = k;
                    rr.pad = 0;
                    rr.c = c;
                    rr.s = s;
                    rots[nrot] = rr;
                }
            }
            ++nrot;
            if (nrot > max_rot) {
                fail = 2;
                break;
            }
        }
        if (fail) break;
    }
    wave_sync();
    // packed upper triangle
    for (int j = 0; j < m; ++j)
        for (int i = lane; i <= j; i += 64) T_out[j * (j + 1) / 2 + i] = H(i, j);
    if (lane == 0) {
        *nrot_out = min(nrot, max_rot);
        *status = fail;
    }
}

// Q = product of the recorded rotations' conjugate transposes, row by row:
// Q(i, :) <- Q(i, :) G_r^H for r = 0 .. nrot-1, starting from Q = I.
__global__ __launch_bounds__(64) void k_schur_q(int m, const Rot* __restrict__ rots, const int* nrot_p, double beta,
                                                cplx* Q, cplx* g, cplx* qlast) {
    extern __shared__ cplx Qs[];          // 64 rows x (m + 1)
    const int ld = m + 1;
    const int li = threadIdx.x;
    const int i = blockIdx.x * 64 + li;
    cplx* q = Qs + li * ld;
    for (int k = 0; k < m; ++k) q[k] = mk((k == i) ? 1.0 : 0.0, 0.0);
    const int nrot = *nrot_p;
    for (int r = 0; r < nrot; ++r) {
        const Rot rr = rots[r];
        const cplx a = q[rr.k], b = q[rr.k + 1];
        q[rr.k] = mk(rr.c * a.re, rr.c * a.im) + b * conj(rr.s);
        q[rr.k + 1] = mk(rr.c * b.re, rr.c * b.im) - a * rr.s;
    }
    if (i < m) {
        for (int k = 0; k < m; ++k) Q[i + (int64_t)k * m] = q[k];
        if (i == 0)
            for (int k = 0; k < m; ++k) g[k] = mk(beta * q[k].re, -beta * q[k].im);
        if (i == m - 1)
            for (int k = 0; k < m; ++k) qlast[k] = q[k];
    }
}

simm_status hess_schur(const cplx* H, int ldh, int m, double beta, SchurOut out, int* status, hipStream_t st) {
    if (m < 1 || m > MAX_SCHUR_M) {
        set_error("Krylov dimension outside 1..128");
        return SIMM_EUNSUPPORTED;
    }
    const int max_rot = 40 * m * m + 64;
    Rot* rots = nullptr;
    int* nrot = nullptr;
    SIMM_HIP_TRY(hipMallocAsync((void**)&rots, sizeof(Rot) * (size_t)max_rot + 256, st));
    nrot = reinterpret_cast<int*>(reinterpret_cast<char*>(rots) + sizeof(Rot) * (size_t)max_rot);
    const size_t lds1 = sizeof(cplx) * (size_t)(m * (m + 5) / 2 + 8);
    hipLaunchKernelGGL(k_hess_qr, dim3(1), dim3(64), lds1, st, H, ldh, m, rots, max_rot, nrot, out.T, status);
    const size_t lds2 = sizeof(cplx) * (size_t)64 * (m + 1);
    hipLaunchKernelGGL(k_schur_q, dim3((m + 63) / 64), dim3(64), lds2, st, m, (const Rot*)rots, (const int*)nrot, beta,
                       out.Q, out.g, out.qlast);
    SIMM_HIP_TRY(hipGetLastError());
    SIMM_HIP_TRY(hipFreeAsync(rots, st));
    return SIMM_OK;
}

}  // namespace simm
