/*
 * simm.h -- C ABI of the MI355X (gfx950) library for the indicator evaluation of
 * SIM-M, the multilevel spectral indicator method for A x = lambda B x
 * (Huang, Sun & Yang, arXiv:2006.16117).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Complex numbers are two interleaved doubles (re, im), i.e. the layout of
 *    C99 double complex / std::complex<double> / numpy complex128.
 *  - Matrices are column-major.  Band matrices use LAPACK general-band layout:
 *    entry (i, j) of an n x n matrix with kl sub- and ku super-diagonals is
 *    band[(ku + i - j) + j * (kl + ku + 1)], for max(0, j-ku) <= i <= min(n-1, j+kl).
 *  - `mem` arguments say where a pointer lives: SIMM_MEM_HOST or SIMM_MEM_DEVICE
 *    (HIP device memory of the current device).
 *  - `hip_stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; unless stated otherwise a call returns after its work has completed.
 *  - Inputs are borrowed for the duration of the call; the library copies what
 *    it keeps.  Objects returned through `out` pointers are library-owned and
 *    must be released with the matching *_destroy call.
 *  - Every call returns a simm_status; no C++ exception crosses the ABI.  On an
 *    error, simm_last_error() returns a description (thread-local, valid until
 *    the next simm_* call on the same thread).
 */
#ifndef SIMM_H
#define SIMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIMM_OK = 0,
    SIMM_EINVAL = -1,           /* bad argument (NaN/Inf input, m < 1, m > n, cap too small, ...) */
    SIMM_ENODEV = -2,           /* no usable gfx950 device */
    SIMM_ENOMEM = -3,           /* device allocation failed */
    SIMM_EHIP = -4,             /* a HIP runtime call failed (message has hipGetErrorString) */
    SIMM_ESINGULAR_SHIFT = -5,  /* exact zero pivot: the shift is an eigenvalue of the pencil */
    SIMM_ENOCONV = -6,          /* the QR iteration for the Schur form of H_m did not converge */
    SIMM_ELIMIT = -7,           /* a level holds more squares than max_regions_per_level */
    SIMM_EUNSUPPORTED = -8,     /* size outside what the kernels support (see each call) */
    SIMM_EREFINE = -9,          /* FP32 factor: iterative refinement did not reach its residual
                                   tolerance (the shift falls back to FP64 inside simm_run) */
    SIMM_EUNRESOLVED = -10      /* simm_gradient: a square's reduced solves (or its adjoint
                                   ones) leave a residual above eps0 (Definition 3.1) */
} simm_status;

enum { SIMM_MEM_HOST = 0, SIMM_MEM_DEVICE = 1 };

/* Region decisions (Definitions 3.1-3.2 and Remark 3.3 of the paper). */
enum { SIMM_REJECTED = 0, SIMM_ADMISSIBLE = 1, SIMM_UNRESOLVED = 2 };

/* simm_params.flags */
enum {
    SIMM_FLAG_PROJECT = 1u,        /* form X = V_m Y for the squares of every level               */
    SIMM_FLAG_KERNEL_TIMING = 2u,  /* bracket every hot-path kernel launch with HIP events        */
    SIMM_FLAG_RELEASE_FACTORS = 4u, /* free every shift's factor, sweep data and Krylov basis when
                                      the run ends (the result keeps the levels, clusters and each
                                      shift's sigma, beta, H and Schur data); simm_shift_apply,
                                      simm_shift_basis and simm_multiplicities on the result then
                                      return EINVAL.  For batches of large pencils.               */
    SIMM_FLAG_MIXED_PROJECT = 8u   /* with SIMM_FLAG_PROJECT: levels 1-2 project in BF16, later
                                      levels in FP32 (FP32 accumulation); every decision, solve
                                      and sum stays FP64, so only the full-space indicator record
                                      (simm_result_full_indicators) changes                       */
};

/* Arithmetic of the shift factors (simm_params.precision, simm_shift_build). */
enum {
    SIMM_PREC_FP64 = 0,            /* band LU and its solves in FP64                               */
    SIMM_PREC_MIXED = 1            /* band LU factored and stored in FP32; every solve with it is
                                      refined against the FP64 pencil until its normwise backward
                                      error ||u - (A - sigma B) x||_inf / (||A - sigma B||_inf
                                      ||x||_inf + ||u||_inf) is at most 1e-12 (at most 2
                                      corrections; SIMM_EREFINE otherwise).  Arnoldi, the Schur
                                      form, the shifted solves, sums and decisions stay FP64; a
                                      run projects in BF16 at levels 1-2 and FP32 after          */
};

/* Arithmetic of simm_project. */
enum {
    SIMM_PROJ_FP64 = 0,            /* FP64 matrix cores                                            */
    SIMM_PROJ_FP32 = 1,            /* V, Y rounded to FP32, FP32 matrix cores, FP32 accumulation   */
    SIMM_PROJ_BF16 = 2             /* V, Y rounded to BF16, FP32 accumulation                      */
};

/* Kernel classes reported by simm_result_kernel_stats. */
enum {
    SIMM_K_BAND_LU = 0,       /* assembly + banded LU of one shift (all its launches)          */
    SIMM_K_BAND_SWEEP = 1,    /* one application of U^{-1} L^{-1} P (its partitioned launches) */
    SIMM_K_GRAM_SCHMIDT = 2,  /* one Arnoldi step's orthogonalisation (its launches)           */
    SIMM_K_SCHUR = 3,         /* Schur form of one H_m                                         */
    SIMM_K_INDICATORS = 4,    /* one indicator launch over a batch of squares                  */
    SIMM_K_PROJECT = 5,       /* one X = V_m Y launch                                          */
    SIMM_K_SPIKE_PREP = 6,    /* per-shift unit-state responses of the partitioned sweeps      */
    SIMM_K_COUNT = 7
};

typedef struct simm_pencil_s* simm_pencil;
typedef struct simm_shift_s* simm_shift;
typedef struct simm_result_s* simm_result;

const char* simm_last_error(void);
int32_t simm_version(void);

/* ------------------------------------------------------------------------ */
/* Pencil (A, B): eq. (AxLambdaBx), A and B n x n, sparse, non-Hermitian.     */
/* ------------------------------------------------------------------------ */

/* Banded A and B in LAPACK band layout (see above).  b_band == NULL means B = I
 * (kl_b, ku_b ignored).  The pencil is copied to device memory.
 * EINVAL: n < 1, negative bandwidths, NULL a_band, NaN/Inf entries. */
simm_status simm_pencil_create_banded(int64_t n,
                                      int32_t kl_a, int32_t ku_a, const double* a_band,
                                      int32_t kl_b, int32_t ku_b, const double* b_band,
                                      int32_t mem, void* hip_stream, simm_pencil* out);

/* CSR A and B (0-based row pointers and column indices, complex values; host
 * memory only).  Converted to band form; b_rowptr == NULL means B = I.
 * EUNSUPPORTED if the half-bandwidth exceeds 4096. */
simm_status simm_pencil_create_csr(int64_t n,
                                   const int64_t* a_rowptr, const int32_t* a_col, const double* a_val,
                                   const int64_t* b_rowptr, const int32_t* b_col, const double* b_val,
                                   void* hip_stream, simm_pencil* out);

simm_status simm_pencil_info(simm_pencil p, int64_t* n, int32_t* kl, int32_t* ku);
/* Shifts and results made on a pencil refer to it (applications of M, Krylov
 * spaces for multiplicities): destroy the pencil after them. */
void simm_pencil_destroy(simm_pencil p);

/* ------------------------------------------------------------------------ */
/* Parameters of SIM-M(A, B, R, f, h0, eps, delta0, m, n0) (Sec. 3.5).       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double x0, x1, y0, y1;      /* search region R = [x0,x1] x [y0,y1]                         */
    int32_t n1;                 /* level-1 cells along x; cells are square, so (y1-y0)/w1 must be
                                   an integer with w1 = (x1-x0)/n1                               */
    int32_t gauss_per_edge;     /* g: the n0-rule has g Gauss-Legendre points per edge, the 2n0-
                                   rule 2g per edge (12 g systems per square)                    */
    int32_t m;                  /* Krylov dimension                                              */
    int32_t levels;             /* K; if <= 0, K = 1 + ceil(log2(w1 / h0))                        */
    double h0;                  /* precision (square width at which refinement stops)            */
    double eps0;                /* residual tolerance of Definition 3.1 (default 1e-8)           */
    double delta0;              /* indicator threshold of Definition 3.2 (default 1/20)          */
    double tau;                 /* floor: admissible needs ||s_f|| > tau * T_f (default 1e-8)    */
    int64_t max_regions_per_level; /* guard against refinement blow-up (default 1<<22)          */
    uint32_t flags;             /* SIMM_FLAG_*                                                   */
    int32_t lookahead;          /* level-1 association: LU factors computed ahead of the cell
                                   order, at most this many at once on streams of their own (0:
                                   one less than GPU_MAX_HW_QUEUES (4 unless set), at most 11;
                                   1: one at a time; at most 16).  Only the shifts the cell order
                                   creates are kept, so results do not depend on it              */
    int32_t precision;          /* SIMM_PREC_FP64 (default) or SIMM_PREC_MIXED.  With MIXED a shift
                                   whose refinement fails (SIMM_EREFINE) is rebuilt with an FP64
                                   factor inside simm_run (counted by simm_result_refine_stats) */
} simm_params;

simm_status simm_params_default(simm_params* p);

/* ------------------------------------------------------------------------ */
/* Hot-path entry points.                                                    */
/* ------------------------------------------------------------------------ */

/* One shift sigma (Sec. 2, Cayley transform and Arnoldi):
 *   banded LU with partial pivoting of A - sigma B (in FP64, or in FP32 with every
 *   solve refined to a backward error of 1e-12: `precision`, SIMM_PREC_*);  b = (A - sigma B)^{-1} f,
 *   beta = ||b||;  m steps of Arnoldi on M = (A - sigma B)^{-1} B from v_1 = b/beta
 *   (classical Gram-Schmidt applied twice), giving V_{m+1}, H_{m+1,m};
 *   then the Schur form H_m = Q T Q^H used by simm_indicators.
 * f: n complex values in `f_mem` memory.  Supported: 1 <= m <= min(n, 128),
 * kl <= 480 of A - sigma B.  Happy breakdown (h_{j+1,j} <= 1e-14 ||M v_j||)
 * stops early with m_eff = j.  ESINGULAR_SHIFT on an exact zero pivot. */
simm_status simm_shift_build(simm_pencil p, double sig_re, double sig_im,
                             const double* f, int32_t f_mem, int32_t m, int32_t precision,
                             void* hip_stream, simm_shift* out);

/* Refined solves of a SIMM_PREC_MIXED shift so far (its Krylov phase, simm_shift_apply):
 * solves, corrections beyond the first solve, and the largest backward error a solve
 * ended with (zeros for an FP64 shift).  Any pointer may be NULL. */
simm_status simm_shift_refine_stats(simm_shift s, int64_t* solves, int64_t* corrections, double* max_eta);

/* How the shift's factor of A - sigma B (Sec. 2, the one factorization per shift behind
 * eq. (IMxb)) was formed.  block_len > 0: partitioned (the diagonal blocks of block_len
 * columns factored side by side with partial pivoting inside each block, the couplings
 * solved through the spikes' reduced system); 0: one band LU of the whole matrix.
 * fallback = 1 when a partitioned factor was replaced by the whole-matrix one (a singular
 * diagonal block or reduced system, or a solve's normwise backward error above 1e-13);
 * eta: that backward error of the partitioned FP64 factor (-1 when not measured).  The
 * library partitions bands with kl, ku >= 1 and 2 kl + ku <= 481 of orders that give
 * blocks of at least max(1024, 4 (kl + ku)) rows, with at most 1 + 2048 / (kl + ku)
 * blocks; the environment variable SIMM_LU_PART = 0 turns it off, and a positive value
 * sets the block length (rounded up to a multiple of 16, at least 256 and 2 (kl + ku)).  Any pointer may be NULL. */
simm_status simm_shift_factor_info(simm_shift s, int64_t* block_len, int32_t* fallback, double* eta);

/* A shift made from its small data alone (Sec. 2, eqs. (shiftedLS), (eq:many) and
 * (eq:error)): the reduced solves (I + (sigma - z_j) H_m) y_j = beta e_1, their
 * residuals and the quadrature sums depend only on sigma, beta = ||(A - sigma B)^{-1} f||
 * and the Arnoldi matrix H_{m+1,m}.  H: (m_eff + 1) x m_eff complex, column-major
 * (leading dimension m_eff + 1), upper Hessenberg, host memory, copied.  The Schur form
 * of H_m is computed on the device, as in simm_shift_build.  The shift has no factor
 * and no basis: simm_indicators accepts it; simm_shift_basis, simm_shift_apply,
 * simm_project and simm_gradient return EINVAL on it.
 * EINVAL: H NULL, NaN/Inf entries, nonzero entries below the subdiagonal, beta not > 0,
 * m_eff < 1; EUNSUPPORTED: m_eff > 128; ENOCONV if the QR iteration fails. */
simm_status simm_shift_from_hessenberg(double sig_re, double sig_im, double beta, const double* H, int32_t m_eff,
                                       void* hip_stream, simm_shift* out);

/* Copies out sigma (2 doubles), beta, m_eff, and optionally (if non-NULL)
 * H_{m_eff+1, m_eff} (column-major complex, leading dimension m_eff+1, host)
 * and the m_eff Ritz values sigma + 1/theta_k (theta_k = eigenvalues of H_m,
 * the diagonal of T; host). */
simm_status simm_shift_info(simm_shift s, double* sigma, double* beta, int32_t* m_eff,
                            double* H, double* ritz);

/* Copies the Arnoldi basis V_{m_eff+1} (n x (m_eff+1), column-major complex,
 * leading dimension n) to `V` in `mem` memory. */
simm_status simm_shift_basis(simm_shift s, double* V, int32_t mem, void* hip_stream);

/* Applies M = (A - sigma B)^{-1} B of this shift to x (n complex): y = M x.
 * x and y in `mem` memory (distinct buffers). */
simm_status simm_shift_apply(simm_shift s, const double* x, double* y, int32_t mem, void* hip_stream);

/* Applies M to k vectors (Sec. 2, eq. (IMxb)): Y(:, r) = M X(:, r), r < k.  X and Y are
 * n x k, column-major complex (leading dimension n), in `mem` memory, distinct buffers.
 * Up to four columns share each pass over the factor; every column equals what
 * simm_shift_apply gives for it.  Synchronous.  EINVAL: bad arguments, k < 0, the
 * factor released; EHIP on a chain time-out. */
simm_status simm_shift_apply_many(simm_shift s, const double* X, double* Y, int32_t k, int32_t mem,
                                  void* hip_stream);

void simm_shift_destroy(simm_shift s);

/* Indicators of N squares (Sec. 2 eqs. (many), (error), (y); Sec. 3.1 eq.
 * (DeltaSm); Definitions 3.1-3.2).  regions: N x 4 int64 rows
 * (level k >= 1, ix, iy, shift index into `shifts`); the square has width
 * w_k = ((x1-x0)/n1) * 2^(1-k) and centre (x0 + (ix+0.5) w_k, y0 + (iy+0.5) w_k).
 * For every one of its 12 g quadrature points z_j the kernel solves
 * (I + (sigma - z_j) H_m) y_j = beta e_1 and forms
 *   rho_j = |sigma - z_j| h_{m+1,m} |e_m^T y_j| / beta,
 *   s_c = (1/2 pi i) sum_{n0-rule} w_j y_j,  s_f = (1/2 pi i) sum_{2n0-rule} w_j y_j,
 *   T_f = (1/2 pi) sum_{2n0-rule} |w_j| ||y_j||.
 * Outputs (each N values, `mem` memory, any may be NULL): indicator = ||s_f||/||s_c||,
 * rho_max = max_j rho_j, nsf = ||s_f||, nsc = ||s_c||, Tf, decision (SIMM_* above;
 * resolvable iff rho_max <= eps0; admissible iff ||s_f|| > tau T_f and
 * ||s_f|| > delta0 ||s_c||).  sums (may be NULL): N x 2 x m_max complex, row r holds
 * s_c then s_f of region r (each m_max entries, zero-padded beyond that shift's m_eff).
 * EUNSUPPORTED if gauss_per_edge > 64. */
simm_status simm_indicators(const simm_shift* shifts, int32_t n_shifts,
                            const int64_t* regions, int64_t n_regions, const simm_params* params,
                            double* indicator, double* rho_max, double* nsf, double* nsc, double* Tf,
                            uint8_t* decision, double* sums, int32_t m_max,
                            int32_t mem, void* hip_stream);

/* Largest residual rho_max = max_j rho_j (Sec. 2, eq. (eq:error)) over the 12 g
 * quadrature points of each of N squares of one level for one shift, from
 * H_{m+1,m} alone (no Schur form; what the association of the level-1 cells uses, since
 * Definition 3.1 asks only whether rho_max <= eps0).  With M_j = I + (sigma - z_j) H_m
 * upper Hessenberg, the cofactor of M_j's (1, m) entry is the product of its
 * subdiagonal, so
 *   rho_j = |sigma - z_j|^m h_{m+1,m} prod_{i<m} h_{i+1,i} / |det M_j|,
 * with det M_j by Gaussian elimination with partial pivoting (rho_j = +Inf if M_j is
 * exactly singular, 0 if h_{m+1,m} = 0).  squares: N x 2 int64 rows (ix, iy) of level
 * `level` (>= 1; centres as in simm_indicators); rho_max: N doubles.  Both in `mem`
 * memory.  EINVAL: NULL arguments, level outside 1..60, N < 0, bad region;
 * EUNSUPPORTED: gauss_per_edge > 64. */
simm_status simm_cell_residuals(simm_shift s, int32_t level, const int64_t* squares, int64_t n_squares,
                                const simm_params* params, double* rho_max, int32_t mem, void* hip_stream);

/* Adjoint gradient of the projected-vector norms J = sum_R ||x_R||^2 over the
 * squares R of `regions` (rows as in simm_indicators), where
 * x_R = (1/2 pi i) sum_j w_j (A - z_j B)^{-1} f is the fine-rule (2 n0 points per
 * edge) quadrature of eq. (XLXf), reduced to the shift's Krylov space as
 * x_R = V_m s_f (eq. (reduced)); f is the start vector the shifts were built from.
 * With c_j = w_j / (2 pi i), u_j = (A - z_j B)^{-1} f and
 * lambda_j = (A - z_j B)^{-H} x_R, the derivative of the resolvent gives
 *   dJ/dp                               = -2 Re sum_R sum_j c_j lambda_j^H A1 u_j,
 *   grad_diag[i] = dJ/dRe A_ii + i dJ/dIm A_ii = -2 conj(sum_R sum_j c_j conj(lambda_j,i) u_j,i),
 * for A = A0 + p A1 with the squares held fixed (decisions are piecewise
 * constant in A).  u_j is V_m y_j from the shift; lambda_j comes from a Krylov
 * space of the conjugate-transposed pencil (A^H, B^H) at conj(sigma), started from
 * x_R (one band LU per shift used, one Krylov space of the shift's m per square).
 * a1_band: band of A1 (kl1 sub-, ku1 superdiagonals, the layout of
 * simm_pencil_create_banded); required when dJdp is not NULL, ignored otherwise.
 * J (required) and dJdp (may be NULL) are host doubles.  grad_diag (may be NULL):
 * n complex values, overwritten.  With dJdp and grad_diag both NULL only J is
 * formed (no adjoint work).  a1_band and grad_diag are in `mem` memory.
 * All shifts must share one pencil and hold their factor and basis; squares whose
 * s_f vanishes contribute nothing.  Every square must be resolved by its shift
 * (max_j rho_j <= eps0, Definition 3.1 with eq. (error)), and every square's adjoint
 * Krylov space likewise at the conjugated nodes; otherwise SIMM_EUNRESOLVED (the
 * derivatives would not be accurate: raise m).  EINVAL on bad rows or arguments,
 * EUNSUPPORTED if m_eff > 128 or gauss_per_edge > 64; SIMM_ESINGULAR_SHIFT if
 * conj(sigma) is an exact eigenvalue of the adjoint pencil. */
simm_status simm_gradient(const simm_shift* shifts, int32_t n_shifts, const int64_t* regions,
                          int64_t n_regions, const simm_params* params, int32_t kl1, int32_t ku1,
                          const double* a1_band, double* J, double* dJdp, double* grad_diag,
                          int32_t mem, void* hip_stream);

/* Projection X = V_m Y (eq. (reduced); the full-space vectors of eq. (ISPf)):
 * Y is m_eff x c complex (column-major, leading dimension m_eff), X is n x c
 * complex (leading dimension n); both in device memory.  col_norms (device, may
 * be NULL) receives ||X(:, j)||_2.  X may be NULL when col_norms is not (only the
 * norms are formed; nothing n x c is written).  `precision` is a SIMM_PROJ_*
 * value: FP64 matrix cores, or V and Y rounded to FP32 / BF16 with FP32
 * accumulation (X and the norms are still returned as FP64).
 * EINVAL: c < 0, Y NULL, both X and col_norms NULL, unknown precision, or the
 * shift's basis was released. */
simm_status simm_project(simm_shift s, const double* Y, int64_t c, double* X, double* col_norms,
                         int32_t precision, void* hip_stream);

/* simm_project without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments and results as simm_project, but the call only enqueues its kernels
 * on hip_stream and returns (no synchronisation).  The column-norm partial sums go to
 * a scratch array that the library holds in device memory (one per device, 16 MiB, kept
 * until the process ends): col_norms needs 8 (2 ceil(n/128) + 32) c bytes of it, and
 * a larger request returns EUNSUPPORTED.  Every call on a device shares that array, so
 * calls that overlap on one device (other streams, before the previous call's kernels
 * have finished) race; calls on one stream are ordered.  X alone needs no scratch. */
simm_status simm_project_noalloc(simm_shift s, const double* Y, int64_t c, double* X, double* col_norms,
                                 int32_t precision, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Whole method: SIM-M steps 1-7 (Sec. 3.5).                                 */
/* ------------------------------------------------------------------------ */

/* Runs SIM-M on the pencil with start vector f (n complex, `f_mem` memory).
 * Step 1: first shift at the centre of R.  Steps 2-3: level-1 cells in (iy, ix)
 * order, each tried against the existing shifts nearest-first (ties: lower
 * index); a cell none of them resolves gets a new shift at its centre.
 * Steps 4-5: K levels; a square keeps its parent's shift, falls back to the
 * other shifts nearest-first if that one does not resolve it, and marked
 * squares (admissible or unresolved) are split into four.  Steps 6-7: marked
 * level-K squares are merged into 8-connected clusters; each cluster's
 * eigenvalue is the mean of its members' centres (and, additionally, the Ritz
 * value of its shift that lies in the cluster).  ELIMIT if a level exceeds
 * max_regions_per_level.  The LU factors of level-1 cells that no shift resolves
 * yet are computed ahead on internal streams (params->lookahead); only those the
 * cell order reaches are used, so the result does not depend on it. */
simm_status simm_run(simm_pencil p, const simm_params* params, const double* f, int32_t f_mem,
                     void* hip_stream, simm_result* out);

/* Batched form: simm_run on `count` independent pencils (sizes may differ), with the
 * same results as `count` separate runs.  Steps 1-3 (the shifts and the level-1 cells) of
 * up to `workers` pencils (at most 16) run in flight at once, each on a non-blocking stream of its own
 * (a lookahead of 0 counts as 1 here, the runs in flight already sharing the queues).
 * Then the levels of all pencils are evaluated together (Sec. 3.3: all squares of a
 * level at once): per level one persistent indicator launch over the squares of every
 * pencil and one grouped FP64 projection over every (pencil, shift), each a captured HIP
 * graph replayed per level (and per round of the shift fallback), with launch shapes
 * picked by timed replays and cached per shape class (simm_batch_tuning).  Pencils whose
 * gauss_per_edge, m, flags or precision differ from the first pencil's take their levels
 * one pencil at a time.  params and f hold one entry per pencil (f[i]: n_i complex values,
 * host or device per f_mem); out receives one result per pencil (caller destroys them).
 * With SIMM_FLAG_RELEASE_FACTORS each pencil's factors are freed after its shifts are
 * built (the bases after the levels).  simm_result_stats reports, per pencil, the time
 * of its shift builds plus the whole batch's level phase.  On any failure every result
 * is destroyed and the first failing pencil's status is returned, with its index in
 * simm_last_error. */
simm_status simm_run_batch(const simm_pencil* pencils, const simm_params* params, const double* const* f,
                           int32_t f_mem, int32_t count, int32_t workers, simm_result* out);

/* Launch shapes the batched form's autotuner has picked in this process: the number of
 * cached shape classes (entries), timed tuning rounds so far (trials), and the chosen
 * workgroup counts of the indicator (ind_grid) and projection (proj_grid) launches, up to
 * cap of each (any pointer may be NULL). */
simm_status simm_batch_tuning(int64_t* entries, int64_t* trials, int32_t* ind_grid, int32_t* proj_grid, int64_t cap);

/* Multiplicities of the eigenvalues of a finished run (Sec. 3.4).  For every shift
 * that one of the clusters' level-K squares was tested with, k Krylov spaces
 * K_m(M, (A - sigma B)^{-1} f_i) are built on that shift's factor; the spectral
 * projection P f_i of a cluster is the sum over its squares of V_m s_f (the fine
 * rule's contour sum of eq. (XLXf) in the Krylov space of eq. (reduced), each
 * square with the space of its own shift; shared edges of adjacent squares cancel).
 * The multiplicity of a cluster is the number of singular values of
 * [P f_1 .. P f_k] above rel_tol times the largest; the singular values come from
 * the k x k Gram matrix, so values below about 1e-8 of the largest are at its
 * rounding level.  F: n x k complex, column-major (leading dimension n), in f_mem
 * memory; 1 <= k <= 64; 0 < rel_tol < 1.  mult (int32 per cluster) and sv (k
 * doubles per cluster, descending; may be NULL) are host arrays with room for
 * cap clusters (EINVAL if cap < the number of clusters).  The pencil the run was
 * made on must still exist.  Synchronous on return. */
simm_status simm_multiplicities(simm_result r, const double* F, int32_t k, int32_t f_mem, double rel_tol,
                                void* hip_stream, int32_t* mult, double* sv, int64_t cap);

simm_status simm_result_summary(simm_result r, int32_t* K, int32_t* n_shifts, int64_t* n_clusters,
                                int64_t* n_unresolved);

/* Squares tested at level `level` (1..K), in the order tested: (iy, ix)
 * lexicographic.  Arrays of `cap` entries (host); any may be NULL.  If cap is
 * too small, EINVAL with *n_tested set to the needed count. */
simm_status simm_result_level(simm_result r, int32_t level, int64_t* n_tested,
                              int64_t* ix, int64_t* iy, int32_t* shift, double* indicator,
                              double* rho_max, uint8_t* decision, int64_t cap);

/* Full-space indicators ||V_m s_f|| / ||V_m s_c|| of the squares of `level`, in
 * the order of simm_result_level (needs SIMM_FLAG_PROJECT; NaN otherwise).  The
 * reduced indicator ||s_f|| / ||s_c|| of simm_result_level equals it up to the
 * orthogonality of V_m (Sec. 3.1).  Host array of `cap` entries. */
simm_status simm_result_full_indicators(simm_result r, int32_t level, double* out, int64_t cap);

/* Shift `idx` of the run (borrowed handle, valid until simm_result_destroy). */
simm_status simm_result_shift(simm_result r, int32_t idx, simm_shift* out);

/* Clusters (eigenvalues): lam = mean of member centres, lam_ritz = Ritz value of
 * the cluster's shift inside the cluster (NaN if none), shift index, flags bit 0
 * = contains an unresolved square.  Host arrays of `cap` entries. */
simm_status simm_result_clusters(simm_result r, int64_t* n, double* lam, double* lam_ritz,
                                 int32_t* shift, int32_t* flags, int64_t cap);

/* Phase timings of the run in milliseconds (host wall clock around
 * stream-synchronised phases): [0] shift builds, [1] indicators, [2] projection,
 * [3] total.  Counters: [0] quadrature-point systems solved, [1] square
 * evaluations, [2] applications of M.  Either pointer may be NULL. */
simm_status simm_result_stats(simm_result r, double* ms4, int64_t* counters3);

/* With SIMM_FLAG_KERNEL_TIMING: total milliseconds and number of timed units per
 * kernel class (SIMM_K_*), measured with HIP events recorded around each unit on
 * the stream it runs on (LU factors computed ahead run on streams of their own, so
 * the class totals may add up to more than the run's wall time).  A unit is one
 * bracketed launch group (one application of M, one Arnoldi step, ...), except for
 * SIMM_K_BAND_LU, whose unit is one 16-column panel launch of the LU.  Arrays of
 * SIMM_K_COUNT entries; zeros otherwise. */
simm_status simm_result_kernel_stats(simm_result r, double* ms, int64_t* launches);

/* Refinement of a SIMM_PREC_MIXED run: refined solves, corrections, shifts rebuilt with an
 * FP64 factor after SIMM_EREFINE, and the largest backward error a refined solve ended
 * with.  Any pointer may be NULL; zeros for an FP64 run. */
simm_status simm_result_refine_stats(simm_result r, int64_t* solves, int64_t* corrections, int32_t* fallbacks,
                                     double* max_eta);

void simm_result_destroy(simm_result r);

#ifdef __cplusplus
}
#endif
#endif /* SIMM_H */
