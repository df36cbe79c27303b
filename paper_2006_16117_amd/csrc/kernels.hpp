// Host-side launchers of the HIP kernels (internal to the library).
#pragma once

#include <atomic>
#include <vector>

#include "common.hpp"

namespace simm {

// hipMalloc that, on running out of memory, first does the frees a batch has deferred
// and tries again (capi.hip)
hipError_t device_malloc(void** p, size_t bytes);
// the stream-ordered form (hipMallocAsync on st; free with hipFreeAsync on st)
hipError_t device_malloc_async(void** p, size_t bytes, hipStream_t st);

// ---- band LU (band_lu.hip) ----
simm_status assemble_shifted(int64_t n, int kl, int ku, const cplx* A, int kla, int kua, const cplx* B, int klb,
                             int kub, cplx sigma, cplx* AB, hipStream_t st);
int lu_panel_width(int kl);
// Permuted multipliers of every 16-column panel (column-major (NB + kl) x NB per panel).
size_t band_lu_panel_elems(int64_t n, int kl);
// info must hold INT_MAX on entry; it receives the first singular column + 1.
// With `cancel`, the launches are enqueued a few hundred at a time and enqueuing
// stops (SIMM_ECANCELED, the factor left incomplete) once *cancel is set.
// `launches` (may be NULL) receives the number of panel launches enqueued.
// bs > 0 (a multiple of 16, below n): the matrix is taken as block diagonal with
// diagonal blocks of bs columns (the last one shorter), each factored on its own, all in
// the same launches; the band must hold zeros outside the blocks.  The result is the
// LU (pivots as global rows) that the whole-matrix factorization gives for such a matrix.
simm_status band_lu(int64_t n, int kl, int ku, cplx* AB, int* ipiv, cplx* LP, int* info, hipStream_t st,
                    const std::atomic<bool>* cancel = nullptr, int64_t* launches = nullptr, int64_t bs = 0);
// the same factorization in FP32 arithmetic and storage (the mixed-precision factor)
simm_status band_lu(int64_t n, int kl, int ku, cplxf* AB, int* ipiv, cplxf* LP, int* info, hipStream_t st,
                    const std::atomic<bool>* cancel = nullptr, int64_t* launches = nullptr, int64_t bs = 0);
simm_status assemble_shifted(int64_t n, int kl, int ku, const cplx* A, int kla, int kua, const cplx* B, int klb,
                             int kub, cplx sigma, cplxf* AB, hipStream_t st);

// ---- input of the sweeps (band_sweep.hip) ----
simm_status prepare_input(int64_t n, const cplx* x, const cplx* Bb, int klb, int kub, const double* hdiv,
                          const int* active, cplx* u, cplx* xs, hipStream_t st);

// ---- partitioned band sweeps (band_spike.hip) ----
// The sweeps run over n16 = n rounded up to 16 (the factor extended by identity),
// in panels of 16 columns.  Per panel they use the blocks below (column-major, so
// that one load instruction reads one column for 64 consecutive rows), formed once
// per shift (spike_prepare):
//   forward  Gf[p] (16 + kl) x 16: rows 0..15 = L11^{-1}, rows 16.. = -L21 L11^{-1}
//            (L = the panel's permuted multipliers),
//   backward Hb[p] (K + 16) x 16: rows 0..K-1 = -U(j0-K .. j0-1, panel) U11^{-1},
//            rows K.. = U11^{-1}.
template <typename GT>      // storage of the per-panel blocks and unit-state responses
struct SpikeFwdT {
    using storage = GT;
    int64_t n, n16;
    int kl;
    const int* ipiv;   // n16 entries (identity past n)
    const GT* G;       // forward panel blocks
    int64_t s;         // chunk length (multiple of 16)
    int mode;          // 0: zero state, input u; 1: unit state blockIdx.y, zero input
    const cplx* u;
    cplx* y;
    cplx* tau;
    GT* Psi;           // n16 x kl
    cplx* Phi;
    const int* active;
    // mode 0 with several right-hand sides (the kernel's NR): column r of u, y and tau
    // at u + r ldu, y + r ldy, tau + r ldt
    int64_t ldu, ldy, ldt;
};
template <typename GT>
struct SpikeBwdT {
    using storage = GT;
    int64_t n, n16;
    int K;
    const GT* H;       // backward panel blocks
    int64_t s;
    int mode;
    const cplx* z;
    cplx* y;
    cplx* tau;
    GT* Psi;           // n16 x K
    cplx* Phi;
    const int* active;
    int64_t ldu, ldy, ldt;   // as in SpikeFwdT (ldu: of z)
};
using SpikeFwd = SpikeFwdT<cplx>;
using SpikeBwd = SpikeBwdT<cplx>;
struct SpikeChain {
    int64_t n;
    int K;
    int64_t P;
    int64_t L;            // chunks per group (groups = gridDim.y); L = P: one group
    int forward;
    const cplx* Phi;
    const cplx* tau;
    cplx* t;
    cplx* gout;           // state after each group's last chunk (groups but the last)
    const cplx* init_src;
    int64_t init_row0;
    unsigned* counter;    // one per group
    int* err;
    const int* active;
    // several right-hand sides (the kernel's NR): state r of t and tau at + r ldt, of
    // gout at + r ldg, of init_src at + r ldi
    int64_t ldt, ldg, ldi;
};
struct SpikeFactor {
    int64_t n = 0, n16 = 0;
    int kl = 0, ku = 0;       // bandwidths of A - sigma B
    cplx* AB = nullptr;       // band LU factor, followed by one zero entry
    int* ipiv = nullptr;      // n16 entries
    const cplx* LP = nullptr; // permuted panel multipliers of the LU
    int K = 0, klx = 0;       // effective upper bandwidth of U, lower bandwidth used
    int64_t s = 0, P = 0;     // chunk length and count
    int Wf = 0, Wb = 0;       // threads of the forward / backward chunk kernels
    void* mem = nullptr;
    cplx *Gf = nullptr, *Hb = nullptr;
    cplx *PsiL = nullptr, *PhiL = nullptr, *PsiU = nullptr, *PhiU = nullptr;
    // FP32 factor (mixed precision): the factor, its panel multipliers, the per-panel
    // blocks and the unit-state responses are stored in FP32 (the blocks and responses
    // formed in FP64 arithmetic from the FP32 factor); the sweeps compute in FP64, and the
    // small per-chunk data (Phi, states, transfer products) stays FP64
    bool f32 = false;
    const cplxf* AB32 = nullptr;
    const cplxf* LP32 = nullptr;
    cplxf *Gf32 = nullptr, *Hb32 = nullptr, *PsiL32 = nullptr, *PsiU32 = nullptr;
    cplx *tauL = nullptr, *tL = nullptr, *tauU = nullptr, *tU = nullptr, *z = nullptr;
    // two-level chain: G groups of L chunks (in chain order); per direction the products
    // Pi_q of the transfer matrices from the start of q's group to chunk q (chain order),
    // the whole-group products, the group outputs and the true group start states
    int64_t G = 1, L = 0;
    cplx *PiL = nullptr, *PiU = nullptr, *PiFullL = nullptr, *PiFullU = nullptr;
    cplx *goutL = nullptr, *goutU = nullptr, *tgL = nullptr, *tgU = nullptr;
    unsigned* counter = nullptr;   // G + 1 counters
    int* err = nullptr;
    // right-hand sides the per-application scratch above holds (z, tau*, t*, gout*, tg*
    // in nrhs slabs each); applications with several at once: spike_apply_diag_nr
    int nrhs = 1;
    // partitioned factorization (band_part.hip): A - sigma B = D + E with D block diagonal
    // (diagonal blocks of bs columns, the last one shorter) and E the couplings of
    // neighbouring blocks; the factor above is D's.  A solve is g = D^{-1} u, the reduced
    // system of the spike tips z = R^{-1} tips(g), and y = g - V t - W b.
    int64_t bs = 0, nbk = 0;       // block length (0: not partitioned) and block count
    int pkl = 0, pku = 0;          // kl, ku of A - sigma B (widths of the couplings)
    int64_t nr = 0;                // order of the reduced system, (nbk - 1)(pkl + pku)
    const cplx* cpl = nullptr;     // couplings per boundary: pku x pku (above), pkl x pkl (below)
    cplx* Vs = nullptr;            // n16 x pku: D^{-1} (upper couplings), column-major
    cplx* Ws = nullptr;            // n16 x pkl: D^{-1} (lower couplings), column-major
    cplx* Rinv = nullptr;          // nr x nr, by rows: the reduced system's inverse
    cplx* pg = nullptr;            // n16: D^{-1} u of an application
    cplx* pz = nullptr;            // nr : the tips of the solution
    void* part_mem = nullptr;
};
int64_t spike_chunk_len(int64_t n, int kl, int K);
simm_status spike_prepare(SpikeFactor& f, hipStream_t st);
simm_status spike_apply(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st);
// an application with D's factor alone (the whole factor when not partitioned)
simm_status spike_apply_diag(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st);
// the same for nr right-hand sides at once (columns u + r ldu -> y + r ldy, r < nr), each
// column computed exactly as spike_apply_diag computes it; nr <= f.nrhs and
// nr <= spike_max_nrhs(f)
simm_status spike_apply_diag_nr(const SpikeFactor& f, const cplx* u, int64_t ldu, cplx* y, int64_t ldy, int nr,
                                hipStream_t st);
// right-hand sides (1, 2 or 4) the chunk kernels of this factor take at once within the LDS
int spike_max_nrhs(const SpikeFactor& f);
// Device-wide budget of the chains' spinning workgroups (band_spike.hip): a phase that
// launches chains holds its weight from before its first launch until its stream is
// done (release synchronizes the stream).  Weight of one stream's applications of f, in
// half compute units, and the budget.
int spike_chain_weight(const SpikeFactor& f);
int spike_chain_budget();
struct ChainSlots {
    int dev = 0, w = 0;
    hipStream_t st = nullptr;
    ChainSlots() = default;
    ChainSlots(const ChainSlots&) = delete;
    ChainSlots& operator=(const ChainSlots&) = delete;
    simm_status acquire(int weight, hipStream_t s);   // blocks the host until the weight is free
    void release();
    ~ChainSlots() { release(); }
};

// ---- partitioned factorization (band_part.hip) ----
constexpr int64_t kPartMaxReduced = 2048;   // largest reduced order (its inverse is nr^2 entries)
// block length of the partitioned factorization of an order-n band (0: factor it whole)
int64_t part_block_len(int64_t n, int kl, int ku);
// copies the couplings of the diagonal blocks out of the assembled band (into cpl,
// nbk - 1 boundaries of ku^2 + kl^2 entries) and zeroes them there
simm_status part_cut(int64_t n, int kl, int ku, cplx* AB, int64_t bs, cplx* cpl, hipStream_t st);
simm_status part_cut(int64_t n, int kl, int ku, cplxf* AB, int64_t bs, cplx* cpl, hipStream_t st);
size_t part_cpl_elems(int64_t n, int kl, int ku, int64_t bs);
// spikes, the reduced system and its inverse of a prepared D factor (f.bs, f.cpl set)
simm_status part_prepare(SpikeFactor& f, hipStream_t st);
simm_status part_apply(const SpikeFactor& f, const cplx* u, cplx* y, const int* active, hipStream_t st);
simm_status part_apply_nr(const SpikeFactor& f, const cplx* u, int64_t ldu, cplx* y, int64_t ldy, int nr,
                          hipStream_t st);
// nr applications at once of the whole factor (partitioned or not): columns u + r ldu ->
// y + r ldy, each as spike_apply computes it; needs nr <= f.nrhs, nr <= spike_max_nrhs(f)
simm_status spike_apply_nr(const SpikeFactor& f, const cplx* u, int64_t ldu, cplx* y, int64_t ldy, int nr,
                           hipStream_t st);
// four streams of a per-device pool made on first use and kept for the process (each
// call takes the next four in turn); callers order their work on them with events
simm_status spike_streams(hipStream_t* out);
void spike_release(SpikeFactor& f);
// ordered = true: the scratch comes from the stream-ordered allocator on st and must be
// freed with spike_release_ordered on st
simm_status spike_clone_scratch(const SpikeFactor& base, SpikeFactor& out, hipStream_t st, bool ordered = false,
                                int nrhs = 1);
void spike_release_ordered(SpikeFactor& f, hipStream_t st);
int64_t spike_bytes_per_apply(const SpikeFactor& f);

// ---- mixed precision: FP64-residual refinement of FP32-factor solves (refine.hip) ----
constexpr double kRefineTol = 1e-12;   // normwise backward error of every refined solve
// corrections before the solve counts as failed.  Every step's kernels are enqueued
// (a device flag skips them once the solve has converged), so each allowed step costs
// its launches on every solve: one correction is what the workloads need.
constexpr int kRefineMaxSteps = 2;
struct RefinePencil {                  // the FP64 shifted pencil the residuals are taken with
    const cplx* A;
    int kla, kua;
    const cplx* B;                     // nullptr: B = I
    int klb, kub;
    cplx sigma;
    double cnorm;                      // ||A - sigma B||_inf
};
struct RefineState {                   // device memory of one shift's refined solves
    cplx* r;                           // n: residual
    cplx* d;                           // n: correction
    unsigned long long* norms;         // [0..2] ||r||, ||x||, ||u|| (inf, as bits); [3] largest final eta
    int* flags;                        // [0] refinement active, [1] tolerance not reached (sticky)
    long long* stats;                  // [0] refined solves, [1] corrections
};
simm_status band_inf_norm(int64_t n, const cplx* A, int kla, int kua, const cplx* B, int klb, int kub, cplx sigma,
                          unsigned long long* scratch, double* host, hipStream_t st);
simm_status refine_apply(const SpikeFactor& f, const RefinePencil& pen, const RefineState& rs, const cplx* u, cplx* y,
                         const int* active, hipStream_t st);
// normwise backward error ||u - C x||_inf / (||C||_inf ||x||_inf + ||u||_inf) of one solve
// x = C^{-1} u with the factor f (u a fixed dense vector; pen.cnorm = ||C||_inf); synchronous
simm_status solve_backward_error(const SpikeFactor& f, const RefinePencil& pen, double* eta, hipStream_t st);
constexpr double kPartTol = 1e-13;     // largest backward error accepted from a partitioned factor
__global__ void k_fill_u64(unsigned long long* p, int count);

// ---- Gram-Schmidt (arnoldi.hip) ----
struct ArnoldiWork {
    int nblk;            // row blocks of the reduction kernels
    cplx* partial;       // nblk x (m + 2)
    cplx* h1;            // m + 2
    cplx* h2;            // m + 2
    double* hnorm;       // device scalars: [0] ||w||, [1] ||M v_j|| (before orthogonalisation)
    cplx* u;             // n   : input of the sweep
};
simm_status arnoldi_step(int64_t n, cplx* V, int64_t ldv, int j, cplx* H, int ldh, ArnoldiWork& w, int* active,
                         int* m_eff, hipStream_t st);
simm_status vec_norm_scale(int64_t n, const cplx* b, cplx* v1, double* beta, ArnoldiWork& w, hipStream_t st);
// per-space pointers of up to four Arnoldi processes advanced together
struct GsBatch {
    cplx* V[4];
    cplx* H[4];
    cplx* partial[4];
    cplx* h1[4];
    cplx* h2[4];
    double* hnorm[4];
    int* active[4];
    int* m_eff[4];
};
simm_status arnoldi_step_batch(int64_t n, const GsBatch& b, int nr, int64_t ldv, int j, int ldh, int nblk,
                               hipStream_t st);

// ---- Schur form of H_m (schur.hip) ----
struct SchurOut {
    cplx* T;       // packed upper triangle by columns: T(i,j) at j(j+1)/2 + i
    cplx* Q;       // m x m column-major
    cplx* g;       // beta * conj(Q(0,:))  (= beta Q^H e_1)
    cplx* qlast;   // Q(m-1, :)
};
simm_status hess_schur(const cplx* H, int ldh, int m, double beta, SchurOut out, int* status, hipStream_t st);

// ---- indicators (indicators.hip) ----
struct ShiftDev {        // per-shift data consumed by the indicator kernel (device memory)
    const cplx* T;
    const cplx* Q;
    const cplx* g;
    const cplx* qlast;
    double sig_re, sig_im;
    double beta;
    double h_last;
    int m;
    int pad;
};
struct RuleDev {         // Gauss-Legendre nodes/weights on [-1, 1] (device memory)
    const double* t1;    // g nodes
    const double* w1;
    const double* t2;    // 2g nodes
    const double* w2;
    int g;
};
struct IndicatorParams {
    double x0, y0, w1;
    double eps0, delta0, tau;
};
// rbits[c] = the largest residual (eq. (error)) over the 12g points of level-`level`
// cell c = (cells[2c], cells[2c+1]) for the shift (sigma, H (ldh, m columns), h_{m+1,m}),
// from Hessenberg determinants (no Schur form); non-negative doubles as bit patterns
simm_status cells_resid(const cplx* H, int ldh, int m, double hlast, cplx sigma, const int64_t* cells, int64_t ncell,
                        int level, const IndicatorParams& prm, const RuleDev& rule, unsigned long long* rbits,
                        hipStream_t st);
simm_status indicators(const ShiftDev* shifts_dev, int mmax, const int64_t* regions, int64_t nreg,
                       const IndicatorParams& prm, const RuleDev& rule, double* indicator, double* rho_max,
                       double* nsf, double* nsc, double* Tf, uint8_t* decision, cplx* sums, int m_sums,
                       hipStream_t st);

// persistent form over the squares of many pencils: rows (level, ix, iy, shift, geometry)
// x nrows[0] (device), geo[] per geometry; grid workgroups take rows in turn
simm_status indicators_persist(const ShiftDev* shifts_dev, int mmax, const int64_t* rows, const int64_t* nrows,
                               const IndicatorParams* geo, const RuleDev& rule, int grid, double* indicator,
                               double* rho_max, double* nsf, double* nsc, double* Tf, uint8_t* decision, cplx* sums,
                               int m_sums, hipStream_t st);

// ---- multiplicities (multiplicity.hip) ----
simm_status cluster_sums(const cplx* sums, int m_sums, const int64_t* off, const int64_t* idx, int64_t ncl,
                         int mrows, cplx* Y, int64_t ldy, hipStream_t st);
simm_status accum_cols(int64_t n, int64_t ncl, const cplx* T, cplx* X, int64_t ldx, hipStream_t st);
// G: ncl x k x k complex, block c column-major k x k: G(a, b) = X_{ck+a}^H X_{ck+b}
simm_status gram(int64_t n, int k, int64_t ncl, const cplx* X, cplx* G, hipStream_t st);
std::vector<double> hermitian_eigenvalues(int k, const cplx* G);

// fine-rule solutions y_j = Q yhat_j of one square, one row of Y per node (ldy >= m);
// conj_nodes: conjugated nodes (a shift of the conjugate-transposed pencil); cw: c_j;
// rho (may be null): the residual of each node's reduced solve (8 g values)
simm_status fine_solutions(const ShiftDev& sh, const IndicatorParams& prm, const RuleDev& rule, int level, int64_t ix,
                           int64_t iy, bool conj_nodes, cplx* Y, int ldy, cplx* cw, double* rho, hipStream_t st);

// ---- adjoint gradient (gradient.hip) ----
simm_status conj_transpose_band(int64_t n, int kl, int ku, const cplx* in, cplx* out, hipStream_t st);
simm_status grad_kmat(int nf, const cplx* Yf, const cplx* Ya, int ldy, const cplx* cw, int mf, int ma, cplx* K,
                      hipStream_t st);
// grad (if non-null) += -2 conj(rowsum(conj(V') o Z)); acc[0] += ||x||^2,
// acc[1] += -2 Re sum(conj(V') o Z1) (Z1 may be null); part: grad_part_elems(n)
simm_status grad_rowdot(int64_t n, int ma, const cplx* Vp, int64_t ldv, const cplx* Z, const cplx* Z1, int64_t ldz,
                        const cplx* x, cplx* grad, cplx* part, double* acc, hipStream_t st);
int64_t grad_part_elems(int64_t n);
// grad = sum of the W per-worker gradients (n each, worker order); acc[0..1] += acc[2w..2w+1]
simm_status grad_combine(int64_t n, int W, const cplx* grads, cplx* grad, double* acc, hipStream_t st);

// ---- projection (project.hip) ----
simm_status project(int64_t n, int m, const cplx* V, int64_t ldv, const cplx* Y, int64_t ldy, int64_t c, cplx* X,
                    double* col_norms, double* scratch, int64_t scratch_elems, int prec, hipStream_t st);
// nb independent FP64 products X_b = V_b Y_b (b < nb), operands offset by the given strides
// (in complex elements, any sign); no column norms
simm_status project_batched(int64_t n, int m, const cplx* V, int64_t ldv, int64_t sV, const cplx* Y, int64_t ldy,
                            int64_t sY, int64_t c, cplx* X, int64_t sX, int nb, hipStream_t st);
int64_t project_scratch_elems(int64_t n, int64_t c);
// One product X_g = V_g Y_g of a grouped projection (column norms only; device table).
struct ProjGroup {
    int64_t n;
    int m;
    const cplx* V;
    int64_t ldv;
    const cplx* Y;
    int64_t ldy;
    int64_t c;
    double* colpart;     // (2 gx) x c per-64-row partial sums
    double* part;        // 32 x c
    double* norms;       // c column norms
    int64_t gx, gy;      // row and column blocks (project_group_shape)
};
void project_group_shape(ProjGroup& g);
// every group of the device table (count ngroups[0], at most gz x ... groups), FP64, by
// persistent launches of `grid` workgroups; colpart needs project_scratch_elems(n, c)
simm_status project_groups(const ProjGroup* groups, const int64_t* ngroups, int grid, int gz, hipStream_t st);

}  // namespace simm
