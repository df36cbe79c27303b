// Projection X = V_m Y of the quadrature sums back to C^n (Sec. 2, eq. (reduced);
// the full-space vectors P_R f of the RIM-C indicator, eq. (ISPf)).
//
// Complex GEMM on the FP64 matrix cores through a real embedding: with a real
// inner index (k, p) (complex index k, part p) and real output columns (j, o),
//   X_real(i, (j,o)) = sum_{(k,p)} V_real(i, (k,p)) Ybig((k,p), (j,o)),
//   Ybig = [[Yr, Yi], [-Yi, Yr]]  (per (k, j) 2x2 block),
// i.e. 8 n m c real flops.  The instruction v_mfma_f64_16x16x4f64 computes X^T
// tiles: its 16 output columns are 16 consecutive rows i of X, so every lane ends
// up with both parts of X(i, j) for two columns j and stores 16-byte complex
// values, contiguous across lanes.
//
// Tiling: a workgroup of four wavefronts owns a 128 x 64 (complex) block of X; each
// wavefront a 64 x 32 block, i.e. 4 x 4 instruction tiles held in 16 accumulators,
// so every operand read from LDS feeds four instructions.  The inner dimension is
// staged through LDS 8 complex indices at a time (double-buffered, the next stage
// loaded into registers while the current one is multiplied).  Each lane reads one
// complex value per operand and uses its real part in one 4-deep step and its
// imaginary part in the next.  Blocks are ordered so that each XCD (workgroups are
// dealt to the eight XCDs in turn) walks a contiguous range of row blocks, all
// column blocks of a row block in a row: that row block of V stays in the XCD's L2.
//
// Reduced-precision forms (the projections of the coarse levels only feed the
// full-space indicator record, never a decision): FP32 operands on
// v_mfma_f32_16x16x4f32 with FP32 accumulation, and BF16 operands on
// v_mfma_f32_16x16x16bf16_1k with FP32 accumulation (16 real inner indices per
// instruction: lane group g supplies (re, im) of the complex indices 2g and 2g + 1
// of the stage).  V and Y stay FP64 in memory and are rounded when read from LDS;
// X is written as complex128.  With X == NULL only the column norms are formed.
#include "common.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace simm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));   // (re, im) in LDS: selects stay on values
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// FP64 -> BF16, round to nearest even (finite inputs)
__device__ inline short to_bf16(double x) {
    const unsigned u = __float_as_uint((float)x);
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

constexpr int PJ_THREADS = 256;
constexpr int PJ_ROWS = 128;            // rows of X per workgroup (2 wavefronts x 64)
constexpr int PJ_COLS = 64;             // complex columns of X per workgroup (2 wavefronts x 32)
constexpr int PJ_KC = 8;                // complex inner indices per LDS stage
constexpr int PJ_YLD = PJ_COLS + 1;     // padded LDS row of a Y stage (conflict-free staging writes)
constexpr int PJ_XCDS = 8;

}  // namespace

// LDS stages of one tile
struct VmyShared {
    d2 Vs[2][PJ_KC][PJ_ROWS];
    d2 Ys[2][PJ_KC][PJ_YLD];
};

// Tile t (row block t / gy, column block t % gy) of X = V Y: the 128 x 64 block of X and
// its per-64-row partial column norms.  Ends with a workgroup barrier.
template <int PREC>
__device__ __forceinline__ void vmy_tile(int64_t n, int m, const cplx* __restrict__ V, int64_t ldv,
                                         const cplx* __restrict__ Y, int64_t ldy, int64_t c, int64_t gy, int64_t t,
                                         cplx* __restrict__ X, double* __restrict__ colpart, VmyShared& sm) {
    auto& Vs = sm.Vs;
    auto& Ys = sm.Ys;
    const int64_t rb = t / gy;
    const int64_t i0 = rb * PJ_ROWS, j0 = (t % gy) * PJ_COLS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, kk = lane >> 4;
    const int wi = wave & 1, wj = wave >> 1;

    // staging: thread -> V rows vr of inner indices vk + 2q (q < 4), Y inner index yk of columns yj + 32q (q < 2)
    const int vr = tid & (PJ_ROWS - 1), vk = tid >> 7;
    const int yk = tid & (PJ_KC - 1), yj = tid >> 3;
    const bool vrow = i0 + vr < n;
    const int64_t vrc = min(i0 + vr, n - 1);
    cplx gv[4], gw[2];
    // loads are unconditional (indices outside the operands are clamped into them) and the
    // values are zeroed afterwards, so that no load sits in a branch
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + vk + 2 * q;
            gv[q] = csel(vrow && k < m, V[vrc + (int64_t)min(k, m - 1) * ldv], mk(0.0, 0.0));
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int k = k0 + yk;
            const int64_t j = j0 + yj + 32 * q;
            gw[q] = csel(k < m && j < c, Y[min(k, m - 1) + min(j, c - 1) * ldy], mk(0.0, 0.0));
        }
    };
    auto stage = [&](int b) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Vs[b][vk + 2 * q][vr] = d2{gv[q].re, gv[q].im};
#pragma unroll
        for (int q = 0; q < 2; ++q) Ys[b][yk][yj + 32 * q] = d2{gw[q].re, gw[q].im};
    };

    // A operand row li of a tile <-> (column of its 8, part).  The FP64 instruction leaves
    // output row r in register r / 4 of lane group r % 4, the FP32-accumulating ones in
    // register r % 4 of lane group r / 4; with the mappings below lane group g then holds
    // (re, im) of columns 2g and 2g + 1 in registers 0..3 in both cases.
    const int ja = (PREC == SIMM_PROJ_FP64) ? 2 * (li & 3) + (li >> 3) : (li >> 1);
    const bool aim = (PREC == SIMM_PROJ_FP64) ? ((li >> 2) & 1) : (li & 1);

    typedef typename std::conditional<PREC == SIMM_PROJ_FP64, d4, f4>::type acc_t;
    acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    fetch(0);
    stage(0);
    __syncthreads();
    const int nch = (m + PJ_KC - 1) / PJ_KC;
    // The loop body has no branch (the stage after the last is fetched as zeros and written to
    // the idle buffer), so the accumulators stay in their registers across iterations.
    for (int ch = 0; ch < nch; ++ch) {
        const int b = ch & 1;
        fetch((ch + 1) * PJ_KC);
        if constexpr (PREC == SIMM_PROJ_BF16) {
            // one instruction per tile and stage: lane group kk supplies the real inner indices
            // (2kk, re), (2kk, im), (2kk+1, re), (2kk+1, im)
            s4 bv[4], av[4];
#pragma unroll
            for (int ti = 0; ti < 4; ++ti) {
                const d2 v0 = Vs[b][2 * kk][wi * 64 + 16 * ti + li];
                const d2 v1 = Vs[b][2 * kk + 1][wi * 64 + 16 * ti + li];
                bv[ti] = s4{to_bf16(v0.x), to_bf16(v0.y), to_bf16(v1.x), to_bf16(v1.y)};
            }
#pragma unroll
            for (int tj = 0; tj < 4; ++tj) {
                const d2 y0 = Ys[b][2 * kk][wj * 32 + 8 * tj + ja];
                const d2 y1 = Ys[b][2 * kk + 1][wj * 32 + 8 * tj + ja];
                // Ybig row (k, re) = (Yr, Yi), row (k, im) = (-Yi, Yr)
                av[tj] = s4{to_bf16(aim ? y0.y : y0.x), to_bf16(aim ? y0.x : -y0.y),
                            to_bf16(aim ? y1.y : y1.x), to_bf16(aim ? y1.x : -y1.y)};
            }
#pragma unroll
            for (int tj = 0; tj < 4; ++tj)
#pragma unroll
                for (int ti = 0; ti < 4; ++ti)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[tj], bv[ti], acc[ti][tj], 0, 0, 0);
        } else {
#pragma unroll
            for (int kg = 0; kg < PJ_KC / 4; ++kg) {
                // lane group kk supplies inner index 4 kg + kk of the stage
                const int kl = 4 * kg + kk;
                d2 vb[4], ya[4];
#pragma unroll
                for (int ti = 0; ti < 4; ++ti) vb[ti] = Vs[b][kl][wi * 64 + 16 * ti + li];
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) ya[tj] = Ys[b][kl][wj * 32 + 8 * tj + ja];
                // real part of the inner index: Ybig row (k, 0) = (Yr, Yi); imaginary part:
                // Ybig row (k, 1) = (-Yi, Yr)
#pragma unroll
                for (int part = 0; part < 2; ++part) {
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj) {
                        const double a = part == 0 ? (aim ? ya[tj].y : ya[tj].x) : (aim ? ya[tj].x : -ya[tj].y);
#pragma unroll
                        for (int ti = 0; ti < 4; ++ti) {
                            const double v = part == 0 ? vb[ti].x : vb[ti].y;
                            if constexpr (PREC == SIMM_PROJ_FP64)
                                acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, v, acc[ti][tj], 0, 0, 0);
                            else
                                acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)v, acc[ti][tj],
                                                                                    0, 0, 0);
                        }
                    }
                }
            }
        }
        stage(b ^ 1);
        __syncthreads();
    }

    // acc[ti][tj]: lane (li, kk), registers (0,1) = X(i, jA), (2,3) = X(i, jA + 1) with
    // i = i0 + 64 wi + 16 ti + li, jA = j0 + 32 wj + 8 tj + 2 kk
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) {
        const int64_t jA = j0 + wj * 32 + 8 * tj + 2 * kk;
        double pa = 0.0, pb = 0.0;
#pragma unroll
        for (int ti = 0; ti < 4; ++ti) {
            const int64_t i = i0 + wi * 64 + 16 * ti + li;
            const cplx xa = mk((double)acc[ti][tj][0], (double)acc[ti][tj][1]);
            const cplx xb = mk((double)acc[ti][tj][2], (double)acc[ti][tj][3]);
            if (i < n) {
                if (X != nullptr) {
                    if (jA < c) X[i + jA * n] = xa;
                    if (jA + 1 < c) X[i + (jA + 1) * n] = xb;
                }
                pa += norm2(xa);
                pb += norm2(xb);
            }
        }
        if (colpart != nullptr) {
            // sum over the 16 lanes li of the group: the wavefront's 64 rows
#pragma unroll
            for (int msk = 8; msk >= 1; msk >>= 1) {
                pa += __shfl_xor(pa, msk, 64);
                pb += __shfl_xor(pb, msk, 64);
            }
            if (li == 0) {
                const int64_t w = 2 * rb + wi;   // 64-row block of X
                if (jA < c) colpart[w * c + jA] = pa;
                if (jA + 1 < c) colpart[w * c + jA + 1] = pb;
            }
        }
    }
}

template <int PREC>
__global__ __launch_bounds__(PJ_THREADS) void k_vmy(int64_t n, int m, const cplx* __restrict__ V, int64_t ldv,
                                                    const cplx* __restrict__ Y, int64_t ldy, int64_t c,
                                                    int64_t gx, int64_t gy, cplx* __restrict__ X,
                                                    double* __restrict__ colpart, int64_t sV, int64_t sY, int64_t sX) {
    // batch member blockIdx.y (strided operands; a batch has no column norms)
    V += (int64_t)blockIdx.y * sV;
    Y += (int64_t)blockIdx.y * sY;
    if (X != nullptr) X += (int64_t)blockIdx.y * sX;
    __shared__ VmyShared sm;
    const int64_t T = gx * gy, per = (T + PJ_XCDS - 1) / PJ_XCDS;
    const int64_t t = (int64_t)(blockIdx.x % PJ_XCDS) * per + blockIdx.x / PJ_XCDS;
    if (t >= T) return;   // uniform over the workgroup
    vmy_tile<PREC>(n, m, V, ldv, Y, ldy, c, gy, t, X, colpart, sm);
}

// Persistent form over groups of products X_g = V_g Y_g (column norms only; the groups
// of a level: one per pencil and shift).  The tile order of every group is that of
// k_vmy (each XCD walks a contiguous range of the group's tiles), workgroup w on XCD
// w % 8 taking every (gridDim.x / 8)-th tile of its XCD's range; a tile's arithmetic is
// that of k_vmy, so the norms equal a launch per group.
__global__ __launch_bounds__(PJ_THREADS) void k_vmy_groups(const ProjGroup* __restrict__ groups,
                                                           const int64_t* __restrict__ ngroups) {
    __shared__ VmyShared sm;
    const int64_t G = *ngroups;
    const int xcd = blockIdx.x % PJ_XCDS;
    const int64_t lw = blockIdx.x / PJ_XCDS, nw = gridDim.x / PJ_XCDS;
    for (int64_t g = 0; g < G; ++g) {
        const ProjGroup gr = groups[g];
        const int64_t T = gr.gx * gr.gy, per = (T + PJ_XCDS - 1) / PJ_XCDS;
        const int64_t t1 = min(T, (int64_t)(xcd + 1) * per);
        for (int64_t t = (int64_t)xcd * per + lw; t < t1; t += nw)
            vmy_tile<SIMM_PROJ_FP64>(gr.n, gr.m, gr.V, gr.ldv, gr.Y, gr.ldy, gr.c, gr.gy, t, nullptr, gr.colpart, sm);
    }
}

// Column norms from the per-64-row-block partial sums: first CN_GROUPS groups of blocks
// each reduce their share for 64 columns (4 threads per column, LDS combine),
// then one pass adds the groups and takes the square root.
constexpr int CN_GROUPS = 32;

__global__ __launch_bounds__(256) void k_colnorm_partial(const double* __restrict__ colpart, int64_t nwaves, int64_t c,
                                                         double* __restrict__ part) {
    __shared__ double red[4][64];
    const int jl = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + jl;
    const int64_t per = (nwaves + CN_GROUPS - 1) / CN_GROUPS;
    const int64_t w0 = (int64_t)blockIdx.y * per, w1 = min(nwaves, w0 + per);
    double a0 = 0.0, a1 = 0.0;
    if (j < c) {
        int64_t w = w0 + sub;
        for (; w + 4 < w1; w += 8) {
            a0 += colpart[w * c + j];
            a1 += colpart[(w + 4) * c + j];
        }
        if (w < w1) a0 += colpart[w * c + j];
    }
    red[sub][jl] = a0 + a1;
    __syncthreads();
    if (sub == 0 && j < c) part[(int64_t)blockIdx.y * c + j] = red[0][jl] + red[1][jl] + red[2][jl] + red[3][jl];
}

__global__ void k_colnorm_finish(const double* __restrict__ part, int64_t c, double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= c) return;
    double acc = 0.0;
    for (int g = 0; g < CN_GROUPS; ++g) acc += part[(int64_t)g * c + j];
    out[j] = sqrt(acc);
}

// The two column-norm reductions of k_colnorm_partial / k_colnorm_finish for every group
// (same order of additions), groups dealt to blockIdx.z in turn.
__global__ __launch_bounds__(256) void k_colnorm_partial_groups(const ProjGroup* __restrict__ groups,
                                                                const int64_t* __restrict__ ngroups) {
    __shared__ double red[4][64];
    const int jl = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int64_t G = *ngroups;
    for (int64_t g = blockIdx.z; g < G; g += gridDim.z) {
        const ProjGroup gr = groups[g];
        const int64_t c = gr.c, nwaves = 2 * gr.gx;
        const int64_t per = (nwaves + CN_GROUPS - 1) / CN_GROUPS;
        const int64_t w0 = (int64_t)blockIdx.y * per, w1 = min(nwaves, w0 + per);
        for (int64_t jb = blockIdx.x; jb * 64 < c; jb += gridDim.x) {
            const int64_t j = jb * 64 + jl;
            double a0 = 0.0, a1 = 0.0;
            if (j < c) {
                int64_t w = w0 + sub;
                for (; w + 4 < w1; w += 8) {
                    a0 += gr.colpart[w * c + j];
                    a1 += gr.colpart[(w + 4) * c + j];
                }
                if (w < w1) a0 += gr.colpart[w * c + j];
            }
            red[sub][jl] = a0 + a1;
            __syncthreads();
            if (sub == 0 && j < c)
                gr.part[(int64_t)blockIdx.y * c + j] = red[0][jl] + red[1][jl] + red[2][jl] + red[3][jl];
            __syncthreads();
        }
    }
}

__global__ void k_colnorm_finish_groups(const ProjGroup* __restrict__ groups, const int64_t* __restrict__ ngroups) {
    const int64_t G = *ngroups;
    for (int64_t g = blockIdx.y; g < G; g += gridDim.y) {
        const ProjGroup gr = groups[g];
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < gr.c; j += (int64_t)gridDim.x * blockDim.x) {
            double acc = 0.0;
            for (int q = 0; q < CN_GROUPS; ++q) acc += gr.part[(int64_t)q * gr.c + j];
            gr.norms[j] = sqrt(acc);
        }
    }
}

int64_t project_scratch_elems(int64_t n, int64_t c) {
    const int64_t nblk64 = 2 * ((n + PJ_ROWS - 1) / PJ_ROWS);   // 64-row blocks of the row-block grid
    return (nblk64 + CN_GROUPS) * c;
}

simm_status project(int64_t n, int m, const cplx* V, int64_t ldv, const cplx* Y, int64_t ldy, int64_t c, cplx* X,
                    double* col_norms, double* scratch, int64_t scratch_elems, int prec, hipStream_t st) {
    if (c <= 0) return SIMM_OK;
    if (prec != SIMM_PROJ_FP64 && prec != SIMM_PROJ_FP32 && prec != SIMM_PROJ_BF16) {
        set_error("unknown projection precision");
        return SIMM_EINVAL;
    }
    if (X == nullptr && col_norms == nullptr) return SIMM_OK;
    if (m < 1 || n < 1) {
        set_error("projection needs n >= 1 and m >= 1");
        return SIMM_EINVAL;
    }
    const int64_t gx = (n + PJ_ROWS - 1) / PJ_ROWS, gy = (c + PJ_COLS - 1) / PJ_COLS;
    const int64_t nblk64 = 2 * gx;
    if (col_norms != nullptr && scratch_elems < (nblk64 + CN_GROUPS) * c) {
        set_error("projection scratch too small");
        return SIMM_EINVAL;
    }
    const int64_t per = (gx * gy + PJ_XCDS - 1) / PJ_XCDS;
    if (per * PJ_XCDS > 0x7fffffff) {
        set_error("projection too large for one launch");
        return SIMM_ELIMIT;
    }
    auto kern = (prec == SIMM_PROJ_FP64) ? k_vmy<SIMM_PROJ_FP64>
                : (prec == SIMM_PROJ_FP32) ? k_vmy<SIMM_PROJ_FP32> : k_vmy<SIMM_PROJ_BF16>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(per * PJ_XCDS)), dim3(PJ_THREADS), 0, st, n, m, V, ldv, Y, ldy, c, gx,
                       gy, X, col_norms ? scratch : nullptr, (int64_t)0, (int64_t)0, (int64_t)0);
    if (col_norms != nullptr) {
        double* part = scratch + nblk64 * c;
        hipLaunchKernelGGL(k_colnorm_partial, dim3((unsigned)((c + 63) / 64), CN_GROUPS), dim3(256), 0, st,
                           (const double*)scratch, nblk64, c, part);
        hipLaunchKernelGGL(k_colnorm_finish, dim3((unsigned)((c + 127) / 128)), dim3(128), 0, st,
                           (const double*)part, c, col_norms);
    }
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

void project_group_shape(ProjGroup& g) {
    g.gx = (g.n + PJ_ROWS - 1) / PJ_ROWS;
    g.gy = (g.c + PJ_COLS - 1) / PJ_COLS;
}
int64_t project_group_scratch(int64_t n, int64_t c) { return project_scratch_elems(n, c); }

simm_status project_groups(const ProjGroup* groups, const int64_t* ngroups, int grid, int gz, hipStream_t st) {
    const int g8 = std::max(PJ_XCDS, grid / PJ_XCDS * PJ_XCDS);
    hipLaunchKernelGGL(k_vmy_groups, dim3((unsigned)g8), dim3(PJ_THREADS), 0, st, groups, ngroups);
    hipLaunchKernelGGL(k_colnorm_partial_groups, dim3(8, CN_GROUPS, (unsigned)gz), dim3(256), 0, st, groups, ngroups);
    hipLaunchKernelGGL(k_colnorm_finish_groups, dim3(4, (unsigned)gz), dim3(128), 0, st, groups, ngroups);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

simm_status project_batched(int64_t n, int m, const cplx* V, int64_t ldv, int64_t sV, const cplx* Y, int64_t ldy,
                            int64_t sY, int64_t c, cplx* X, int64_t sX, int nb, hipStream_t st) {
    if (nb <= 0 || c <= 0) return SIMM_OK;
    if (m < 1 || n < 1 || X == nullptr || nb > 65535) {
        set_error("bad batched projection");
        return SIMM_EINVAL;
    }
    const int64_t gx = (n + PJ_ROWS - 1) / PJ_ROWS, gy = (c + PJ_COLS - 1) / PJ_COLS;
    const int64_t per = (gx * gy + PJ_XCDS - 1) / PJ_XCDS;
    hipLaunchKernelGGL(k_vmy<SIMM_PROJ_FP64>, dim3((unsigned)(per * PJ_XCDS), (unsigned)nb), dim3(PJ_THREADS), 0, st,
                       n, m, V, ldv, Y, ldy, c, gx, gy, X, (double*)nullptr, sV, sY, sX);
    SIMM_HIP_TRY(hipGetLastError());
    return SIMM_OK;
}

}  // namespace simm
