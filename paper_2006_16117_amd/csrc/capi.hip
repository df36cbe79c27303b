// C ABI of the SIM-M library: pencils, shifts, the hot-path entry points and the
// multilevel driver (Sec. 3.3 and the SIM-M algorithm of Sec. 3.5).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <set>
#include <atomic>
#include <chrono>
#include <functional>
#include <string>
#include <thread>
#include <tuple>
#include <utility>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace simm {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

// Frees of the buffers a run releases at its end (SIMM_FLAG_RELEASE_FACTORS).  A free
// waits for the whole device, so while a batch has runs in flight on other streams
// the buffers are collected and freed together once they add up to kDeferBytes (one
// wait instead of one per buffer), and at the end of the batch.
static std::mutex g_free_mu;
static std::vector<void*> g_free_list;
static size_t g_free_bytes = 0;
static std::atomic<int> g_batches{0};
constexpr size_t kDeferBytes = (size_t)16 << 30;

void flush_deferred_frees() {
    std::vector<void*> v;
    {
        std::lock_guard<std::mutex> lk(g_free_mu);
        v.swap(g_free_list);
        g_free_bytes = 0;
    }
    for (void* q : v) (void)hipFree(q);
}

void release_device(void* q) {
    if (!q) return;
    if (g_batches.load() == 0) {
        (void)hipFree(q);
        return;
    }
    size_t bytes = 0;
    if (hipMemPtrGetInfo(q, &bytes) != hipSuccess) bytes = 0;
    bool flush = false;
    {
        std::lock_guard<std::mutex> lk(g_free_mu);
        g_free_list.push_back(q);
        g_free_bytes += bytes;
        flush = g_free_bytes >= kDeferBytes;
    }
    if (flush) flush_deferred_frees();
}

// hipMalloc; when the device is out of memory, the frees collected so far are done
// and the allocation is tried once more.
hipError_t device_malloc(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipErrorOutOfMemory) return e;
    (void)hipGetLastError();
    bool pending;
    {
        std::lock_guard<std::mutex> lk(g_free_mu);
        pending = !g_free_list.empty();
    }
    if (!pending) return e;
    flush_deferred_frees();
    return hipMalloc(p, bytes);
}

constexpr int64_t kGsRowBlocks = 1024;

// hipMallocAsync on st (memory used and freed, with hipFreeAsync, in the order of st, so
// that no device-wide wait is needed), with the same retry as device_malloc.
hipError_t device_malloc_async(void** p, size_t bytes, hipStream_t st) {
    hipError_t e = hipMallocAsync(p, bytes, st);
    if (e != hipErrorOutOfMemory) return e;
    (void)hipGetLastError();
    bool pending;
    {
        std::lock_guard<std::mutex> lk(g_free_mu);
        pending = !g_free_list.empty();
    }
    if (!pending) return e;
    flush_deferred_frees();
    return hipMallocAsync(p, bytes, st);
}

// While one is alive, frees through release_device are collected (runs that release
// their factors shift by shift, batches); the last one to end frees them.
struct DeferFrees {
    bool on;
    explicit DeferFrees(bool enable) : on(enable) {
        if (on) g_batches.fetch_add(1);
    }
    ~DeferFrees() {
        if (on && g_batches.fetch_sub(1) == 1) flush_deferred_frees();
    }
    DeferFrees(const DeferFrees&) = delete;
    DeferFrees& operator=(const DeferFrees&) = delete;
};

}  // namespace simm

using namespace simm;

// ---------------------------------------------------------------------------
// objects
// ---------------------------------------------------------------------------
struct simm_pencil_s {
    int64_t n = 0;
    int kla = 0, kua = 0, klb = 0, kub = 0;
    cplx* A = nullptr;       // device band of A
    cplx* B = nullptr;       // device band of B (nullptr: identity)
    int dev = 0;
};

struct simm_shift_s {
    simm_pencil_s* p = nullptr;
    cplx sigma{0, 0};
    int m = 0, m_eff = 0;
    int kl = 0, ku = 0;
    double beta = 0.0, h_last = 0.0;
    cplx* AB = nullptr;      // LU factor (band)
    int* ipiv = nullptr;     // 16 ceil(n/16) entries (identity past n)
    cplx* LP = nullptr;      // permuted multipliers of every LU panel
    cplx* V = nullptr;       // n x (m+1)
    cplx* H = nullptr;       // (m+1) x m, device
    cplx* T = nullptr;       // packed upper triangle
    cplx* Q = nullptr;       // m_eff x m_eff
    cplx* g = nullptr;
    cplx* qlast = nullptr;
    // mixed precision: FP32 factor (AB32, LP32 instead of AB, LP) whose solves are
    // refined against the FP64 pencil (rpen) with the device state rst (in ref_mem)
    bool mixed = false;
    cplxf* AB32 = nullptr;
    cplxf* LP32 = nullptr;
    RefinePencil rpen{};
    RefineState rst{};
    void* ref_mem = nullptr;
    bool mixed_stats_saved = false;   // refinement counters taken before the factor was freed
    long long saved_stats[2] = {0, 0};
    double saved_eta = 0.0;
    std::vector<cplx> H_host;   // (m_eff+1) x m_eff column-major
    std::vector<cplx> ritz;     // sigma + 1/theta
    bool borrowed = false;      // owned by a simm_result
    bool factor_borrowed = false;   // AB, ipiv, LP, spike belong to another shift
    bool sweeps_ready = false;      // spike holds the partitioned-sweep data of the factor
    SpikeFactor spike;          // partitioned-sweep data of the factor
    // partitioned factorization: block length (0: the whole matrix was factored), the
    // couplings cut from the band, and whether a partitioned factor was replaced by the
    // whole-matrix one (singular block or reduced system, or a backward error above
    // kPartTol, which part_eta records)
    int64_t part_bs = 0;
    cplx* CPL = nullptr;
    // element capacities of V, H and the Schur data: a shift object that builds several
    // Krylov spaces in turn (multiplicities, adjoint spaces) keeps its buffers
    size_t cap_V = 0, cap_H = 0, cap_T = 0, cap_Q = 0, cap_g = 0;
    bool part_fallback = false;
    double part_eta = -1.0;
    // frees the n-sized data (factor, sweep data, Krylov basis); the small per-shift
    // data used by the indicators stays
    void release_large() {
        if (!factor_borrowed) {
            release_device(spike.mem);
            release_device(spike.part_mem);
            release_device(CPL);
            release_device(AB);
            release_device(ipiv);
            release_device(LP);
            release_device(AB32);
            release_device(LP32);
            release_device(ref_mem);
        }
        release_device(V);
        AB = nullptr;
        ipiv = nullptr;
        LP = nullptr;
        AB32 = nullptr;
        LP32 = nullptr;
        ref_mem = nullptr;
        CPL = nullptr;
        V = nullptr;
        cap_V = 0;
        spike = SpikeFactor{};
        factor_borrowed = true;   // nothing left to free
    }
    // frees the factor and its sweep data, keeping the Krylov basis (for the projections)
    void release_factor() {
        if (factor_borrowed) return;
        release_device(spike.mem);
        release_device(spike.part_mem);
        release_device(CPL);
        CPL = nullptr;
        release_device(AB);
        release_device(ipiv);
        release_device(LP);
        release_device(AB32);
        release_device(LP32);
        release_device(ref_mem);
        spike = SpikeFactor{};
        AB = nullptr;
        ipiv = nullptr;
        LP = nullptr;
        AB32 = nullptr;
        LP32 = nullptr;
        ref_mem = nullptr;
        rst = RefineState{};
        mixed_stats_saved = true;
    }
    bool has_factor() const { return (AB != nullptr || AB32 != nullptr) && V != nullptr; }
    // the factor's data for a Krylov space built on it by another (borrowing) shift
    void borrow_factor_of(const simm_shift_s* base) {
        p = base->p;
        sigma = base->sigma;
        kl = base->kl;
        ku = base->ku;
        AB = base->AB;
        ipiv = base->ipiv;
        LP = base->LP;
        mixed = base->mixed;
        AB32 = base->AB32;
        LP32 = base->LP32;
        rpen = base->rpen;
        rst = base->rst;
        spike = base->spike;
        part_bs = base->part_bs;
        CPL = base->CPL;
        sweeps_ready = true;
        factor_borrowed = true;
    }
    // frees through release_device: collected while a run or batch is in flight (a
    // dropped factor computed ahead would otherwise wait for the whole device)
    ~simm_shift_s() {
        if (!factor_borrowed) {
            release_device(spike.mem);
            release_device(spike.part_mem);
            release_device(CPL);
            release_device(AB);
            release_device(ipiv);
            release_device(LP);
            release_device(AB32);
            release_device(LP32);
            release_device(ref_mem);
        }
        release_device(V);
        release_device(H);
        release_device(T);
        release_device(Q);
        release_device(g);
        release_device(qlast);
    }
};

struct LevelRec {
    std::vector<int64_t> ix, iy;
    std::vector<int32_t> shift;
    std::vector<double> indicator, rho_max, nsf, nsc, Tf, full_indicator;
    std::vector<uint8_t> decision;
};

struct ClusterRec {
    cplx lam, lam_ritz;
    int shift;
    int flags;
    std::vector<int64_t> members;   // indices into the last level's squares
};

// HIP-event brackets around kernel launches, collected after the run.
// A bracket counts as one unit unless the code inside sets another count (the LU
// bracket counts its panel launches).
struct KernelClock {
    struct Mark {
        int k;
        hipEvent_t a, b;
        int64_t units;
    };
    hipStream_t st = nullptr;
    std::vector<Mark> marks;
    void begin(int k) {
        hipEvent_t a = nullptr;
        (void)hipEventCreate(&a);
        (void)hipEventRecord(a, st);
        marks.push_back({k, a, nullptr, 1});
    }
    void end(int64_t units) {
        hipEvent_t b = nullptr;
        (void)hipEventCreate(&b);
        (void)hipEventRecord(b, st);
        marks.back().b = b;
        marks.back().units = units;
    }
    void collect(double* ms, int64_t* cnt) {
        for (auto& m : marks) {
            if (m.b) {
                (void)hipEventSynchronize(m.b);
                float t = 0;
                (void)hipEventElapsedTime(&t, m.a, m.b);
                ms[m.k] += t;
                cnt[m.k] += m.units;
                (void)hipEventDestroy(m.b);
            }
            (void)hipEventDestroy(m.a);
        }
        marks.clear();
    }
};

struct KScope {
    KernelClock* c;
    int64_t units = 1;
    KScope(KernelClock* clk, int k) : c(clk) {
        if (c) c->begin(k);
    }
    ~KScope() {
        if (c) c->end(units);
    }
};

struct simm_result_s {
    double kms[SIMM_K_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    int64_t kcnt[SIMM_K_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    double kbytes[SIMM_K_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    int K = 0;
    std::vector<std::unique_ptr<simm_shift_s>> shifts;
    std::vector<LevelRec> levels;
    std::vector<ClusterRec> clusters;
    double ms[4] = {0, 0, 0, 0};
    int64_t counters[3] = {0, 0, 0};
    // mixed precision: refined solves, their corrections, shifts rebuilt in FP64 after a
    // refinement failure, and the largest backward error a refined solve ended with
    int64_t refine_solves = 0, refine_corrections = 0;
    int32_t refine_fallbacks = 0;
    double refine_max_eta = 0.0;
    simm_params prm{};               // the run's parameters
    simm_pencil_s* pencil = nullptr; // borrowed: the pencil the run was made on
};

namespace {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1] by Newton's method on P_g.
void gauss_legendre(int g, std::vector<double>& x, std::vector<double>& w) {
    x.assign(g, 0.0);
    w.assign(g, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (g + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (g + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= g; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (g == 1) {
                p1 = z;
                p0 = 1.0;
            }
            dp = g * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                // one more evaluation at the converged point for the weight
                p0 = 1.0;
                p1 = z;
                for (int k = 2; k <= g; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = g * (z * p1 - p0) / (z * z - 1.0);
                break;
            }
        }
        const double wt = 2.0 / ((1.0 - z * z) * dp * dp);
        x[g - 1 - i] = z;      // z > 0 for small i
        x[i] = -z;
        w[g - 1 - i] = wt;
        w[i] = wt;
    }
    if (g % 2 == 1) x[g / 2] = 0.0;
}

bool finite_c(const double* v, int64_t count) {
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

template <typename T>
simm_status dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = device_malloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SIMM_ENOMEM : SIMM_EHIP;
    }
    return SIMM_OK;
}

// Scratch device buffer, allocated and freed in stream order on the stream of the
// call that uses it (a plain free would wait for the whole device and serialise
// concurrent runs on other streams).  Stream-ordered memory must not outlive the
// stream it was allocated on, so every live buffer is registered with its stream, and
// a stream's owner frees what is still registered on it before destroying the stream
// (release_stream_buffers); the buffer's own destructor then has nothing left to free.
struct DevBuf;
std::mutex g_devbuf_mu;
std::multimap<hipStream_t, DevBuf*> g_devbuf_live;

struct DevBuf {
    void* p = nullptr;
    hipStream_t st = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        std::lock_guard<std::mutex> lk(g_devbuf_mu);
        release_locked();
    }
    void release_locked() {
        if (!p) return;
        (void)hipFreeAsync(p, st);
        p = nullptr;
        auto range = g_devbuf_live.equal_range(st);
        for (auto it = range.first; it != range.second; ++it)
            if (it->second == this) {
                g_devbuf_live.erase(it);
                break;
            }
    }
    simm_status alloc(size_t bytes, hipStream_t stream) {
        release();
        st = stream;
        hipError_t e = hipMallocAsync(&p, bytes ? bytes : 1, st);
        if (e != hipSuccess) {
            p = nullptr;
            set_error(std::string("hipMallocAsync: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? SIMM_ENOMEM : SIMM_EHIP;
        }
        std::lock_guard<std::mutex> lk(g_devbuf_mu);
        g_devbuf_live.emplace(st, this);
        return SIMM_OK;
    }
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

// Frees (in stream order) every buffer still allocated on `st`; called by the owner of
// a stream before hipStreamDestroy, once no thread uses the stream any more.
void release_stream_buffers(hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_devbuf_mu);
    while (true) {
        auto it = g_devbuf_live.find(st);
        if (it == g_devbuf_live.end()) break;
        it->second->release_locked();
    }
}

// The current device's stream-ordered memory pool reuses a block freed on one stream
// for another stream only once the free has run on the device (not on the strength of
// event dependencies between the streams: those the runs make are for ordering work,
// and the pool would otherwise hand a later allocation a block whose free is still
// pending).  Set once per device.
std::mutex g_pool_mu;
std::set<int> g_pool_configured;
void configure_pool() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool_configured.insert(dev).second) return;
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess || !pool) return;
    int off = 0;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolReuseFollowEventDependencies, &off);
    (void)hipMemPoolSetAttribute(pool, hipMemPoolReuseAllowInternalDependencies, &off);
}

simm_status check_device() {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
        set_error("no HIP device");
        return SIMM_ENODEV;
    }
    configure_pool();
    return SIMM_OK;
}

struct Rule {
    DevBuf buf;
    int g = 0;
    RuleDev dev{};
    simm_status make(int g_, hipStream_t st) {
        g = g_;
        std::vector<double> t1, w1, t2, w2;
        gauss_legendre(g, t1, w1);
        gauss_legendre(2 * g, t2, w2);
        std::vector<double> all;
        all.insert(all.end(), t1.begin(), t1.end());
        all.insert(all.end(), w1.begin(), w1.end());
        all.insert(all.end(), t2.begin(), t2.end());
        all.insert(all.end(), w2.begin(), w2.end());
        SIMM_TRY(buf.alloc(all.size() * sizeof(double), st));
        SIMM_HIP_TRY(hipMemcpyAsync(buf.p, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));   // `all` is a host temporary
        double* d = buf.as<double>();
        dev.t1 = d;
        dev.w1 = d + g;
        dev.t2 = d + 2 * g;
        dev.w2 = d + 4 * g;
        dev.g = g;
        return SIMM_OK;
    }
};

ShiftDev shift_dev(const simm_shift_s* s) {
    ShiftDev d;
    d.T = s->T;
    d.Q = s->Q;
    d.g = s->g;
    d.qlast = s->qlast;
    d.sig_re = s->sigma.re;
    d.sig_im = s->sigma.im;
    d.beta = s->beta;
    d.h_last = s->h_last;
    d.m = s->m_eff;
    d.pad = 0;
    return d;
}

// Factor phase of one shift (hot-path steps a1-a2): the shifted band and its LU with
// partial pivoting.  Synchronous on return (the factor may be used next on another
// stream).
// With whole = false the band is factored in diagonal blocks when part_block_len says
// so (the spikes and reduced system follow with the sweep data); a singular block
// falls back to the whole-matrix factorization.
simm_status factor_shift(simm_pencil_s* p, cplx sigma, hipStream_t st, std::unique_ptr<simm_shift_s>& out,
                         KernelClock* clk = nullptr, const std::atomic<bool>* cancel = nullptr,
                         int precision = SIMM_PREC_FP64, bool whole = false) {
    auto s = std::make_unique<simm_shift_s>();
    s->p = p;
    s->sigma = sigma;
    const int64_t n = p->n;
    const int kl = std::max(p->kla, p->klb);
    const int ku = std::max(p->kua, p->kub);
    s->kl = kl;
    s->ku = ku;
    const int ldab = 2 * kl + ku + 1;
    if (lu_panel_width(kl) == 0 || kl + ku + 2 > 1024) {
        set_error("pencil bandwidth outside the supported range (kl <= 480, kl + ku <= 1022)");
        return SIMM_EUNSUPPORTED;
    }
    s->mixed = (precision == SIMM_PREC_MIXED);
    s->part_bs = whole ? 0 : part_block_len(n, kl, ku);
    if (s->part_bs > 0) SIMM_TRY(dalloc(&s->CPL, part_cpl_elems(n, kl, ku, s->part_bs)));
    SIMM_TRY(dalloc(&s->ipiv, (size_t)((n + 15) / 16 * 16)));
    if (s->mixed) {
        SIMM_TRY(dalloc(&s->AB32, (size_t)ldab * n + 1));   // + one zero entry read for out-of-band taps
        SIMM_TRY(dalloc(&s->LP32, band_lu_panel_elems(n, kl)));
        // refinement state: residual and correction vectors, norms, flags, counters
        SIMM_HIP_TRY(hipMalloc(&s->ref_mem, sizeof(cplx) * 2 * (size_t)n + 1024));
        cplx* rb = reinterpret_cast<cplx*>(s->ref_mem);
        s->rst.r = rb;
        s->rst.d = rb + n;
        s->rst.norms = reinterpret_cast<unsigned long long*>(rb + 2 * n);
        s->rst.flags = reinterpret_cast<int*>(s->rst.norms + 8);
        s->rst.stats = reinterpret_cast<long long*>(s->rst.norms + 16);
        hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, s->rst.norms, 24);
        SIMM_HIP_TRY(hipGetLastError());
        s->rpen = RefinePencil{p->A, p->kla, p->kua, p->B, p->klb, p->kub, sigma, 0.0};
        SIMM_TRY(band_inf_norm(n, p->A, p->kla, p->kua, p->B, p->klb, p->kub, sigma, s->rst.norms + 4, &s->rpen.cnorm,
                               st));
    } else {
        SIMM_TRY(dalloc(&s->AB, (size_t)ldab * n + 1));   // + one zero entry read for out-of-band taps
        SIMM_TRY(dalloc(&s->LP, band_lu_panel_elems(n, kl)));
    }
    DevBuf info_buf;
    SIMM_TRY(info_buf.alloc(sizeof(int), st));
    int* info_d = info_buf.as<int>();
    int info = INT_MAX;
    SIMM_HIP_TRY(hipMemcpyAsync(info_d, &info, sizeof(int), hipMemcpyHostToDevice, st));
    if (s->mixed) SIMM_HIP_TRY(hipMemsetAsync(s->AB32 + (size_t)ldab * n, 0, sizeof(cplxf), st));
    else SIMM_HIP_TRY(hipMemsetAsync(s->AB + (size_t)ldab * n, 0, sizeof(cplx), st));
    {
        KScope ks(clk, SIMM_K_BAND_LU);
        simm_status lu;
        if (s->mixed) {
            SIMM_TRY(assemble_shifted(n, kl, ku, p->A, p->kla, p->kua, p->B, p->klb, p->kub, sigma, s->AB32, st));
            if (s->part_bs > 0) SIMM_TRY(part_cut(n, kl, ku, s->AB32, s->part_bs, s->CPL, st));
            lu = band_lu(n, kl, ku, s->AB32, s->ipiv, s->LP32, info_d, st, cancel, &ks.units, s->part_bs);
        } else {
            SIMM_TRY(assemble_shifted(n, kl, ku, p->A, p->kla, p->kua, p->B, p->klb, p->kub, sigma, s->AB, st));
            if (s->part_bs > 0) SIMM_TRY(part_cut(n, kl, ku, s->AB, s->part_bs, s->CPL, st));
            lu = band_lu(n, kl, ku, s->AB, s->ipiv, s->LP, info_d, st, cancel, &ks.units, s->part_bs);
        }
        if (lu != SIMM_OK) return lu;
    }
    SIMM_HIP_TRY(hipMemcpyAsync(&info, info_d, sizeof(int), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    if (info != INT_MAX && s->part_bs > 0) {
        // a zero pivot inside a diagonal block says nothing about A - sigma B itself
        SIMM_TRY(factor_shift(p, sigma, st, out, clk, cancel, precision, true));
        out->part_fallback = true;
        return SIMM_OK;
    }
    if (info != INT_MAX) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "exact zero pivot in column %d of A - sigma B (sigma = %.17g%+.17gi)", info,
                      sigma.re, sigma.im);
        set_error(msg);
        return SIMM_ESINGULAR_SHIFT;
    }
    out = std::move(s);
    return SIMM_OK;
}

// Partitioned-sweep data of a shift's factor (a launch wide enough to fill the
// device).  Synchronous on return.
simm_status prepare_sweeps(simm_shift_s* s, hipStream_t st, KernelClock* clk = nullptr) {
    s->spike.n = s->p->n;
    s->spike.kl = s->kl;
    s->spike.ku = s->ku;
    s->spike.AB = s->AB;
    s->spike.ipiv = s->ipiv;
    s->spike.LP = s->LP;
    s->spike.f32 = s->mixed;
    s->spike.AB32 = s->AB32;
    s->spike.LP32 = s->LP32;
    s->spike.bs = s->part_bs;
    s->spike.cpl = s->CPL;
    simm_status rc;
    {
        KScope ks(clk, SIMM_K_SPIKE_PREP);
        rc = spike_prepare(s->spike, st);
    }
    if (rc != SIMM_OK && !(s->part_bs > 0 && rc == SIMM_ESINGULAR_SHIFT)) return rc;
    bool redo = rc != SIMM_OK;
    if (!redo && s->part_bs > 0 && !s->mixed) {
        // pivoting stays inside the blocks: the partitioned factor is kept only if a
        // solve with it is backward stable (the FP32 one is refined anyway)
        simm_pencil_s* p = s->p;
        RefinePencil pen{p->A, p->kla, p->kua, p->B, p->klb, p->kub, s->sigma, 0.0};
        DevBuf nb;
        SIMM_TRY(nb.alloc(sizeof(unsigned long long) * 4, st));
        SIMM_TRY(band_inf_norm(p->n, p->A, p->kla, p->kua, p->B, p->klb, p->kub, s->sigma,
                               nb.as<unsigned long long>(), &pen.cnorm, st));
        SIMM_TRY(solve_backward_error(s->spike, pen, &s->part_eta, st));
        redo = !(s->part_eta <= kPartTol);
    }
    if (redo) {
        // the whole-matrix factor instead, in place of the partitioned one
        std::unique_ptr<simm_shift_s> w;
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        SIMM_TRY(factor_shift(s->p, s->sigma, st, w, clk, nullptr, s->mixed ? SIMM_PREC_MIXED : SIMM_PREC_FP64, true));
        spike_release(s->spike);
        s->spike = SpikeFactor{};
        std::swap(s->AB, w->AB);
        std::swap(s->AB32, w->AB32);
        std::swap(s->LP, w->LP);
        std::swap(s->LP32, w->LP32);
        std::swap(s->ipiv, w->ipiv);
        std::swap(s->CPL, w->CPL);
        s->part_bs = 0;
        s->part_fallback = true;
        return prepare_sweeps(s, st, clk);
    }
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    s->sweeps_ready = true;
    return SIMM_OK;
}

// p holds at least `need` elements (cap: its current capacity): kept when large enough
template <typename T>
simm_status ensure_dev(T** p, size_t& cap, size_t need) {
    if (*p && cap >= need) return SIMM_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    SIMM_TRY(dalloc(p, need));
    cap = need;
    return SIMM_OK;
}

// Schur phase of one shift (hot-path step a5): the complex Schur form H_m = Q T Q^H of
// the device copy of H (leading dimension ldh, s->m_eff columns), g = beta Q^H e_1,
// the last row of Q, and the Ritz values sigma + 1/theta from the diagonal of T.
// status_dev: one device int, the QR iteration's convergence flag.  schur_launch
// enqueues the kernels on st; schur_finish waits for st and takes the status and the
// Ritz values; schur_phase does both.
simm_status schur_launch(simm_shift_s* s, int ldh, int* status_dev, hipStream_t st, KernelClock* clk = nullptr) {
    const int me = s->m_eff;
    size_t cap_q = s->cap_g;   // g and qlast have the same size
    SIMM_TRY(ensure_dev(&s->T, s->cap_T, (size_t)me * (me + 1) / 2));
    SIMM_TRY(ensure_dev(&s->Q, s->cap_Q, (size_t)me * me));
    SIMM_TRY(ensure_dev(&s->g, s->cap_g, (size_t)me));
    SIMM_TRY(ensure_dev(&s->qlast, cap_q, (size_t)me));
    SchurOut so{s->T, s->Q, s->g, s->qlast};
    KScope ks(clk, SIMM_K_SCHUR);
    return hess_schur(s->H, ldh, me, s->beta, so, status_dev, st);
}

simm_status schur_finish(simm_shift_s* s, const int* status_dev, hipStream_t st) {
    const int me = s->m_eff;
    int schur_status = 0;
    std::vector<cplx> Tp((size_t)me * (me + 1) / 2);
    SIMM_HIP_TRY(hipMemcpyAsync(&schur_status, status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipMemcpyAsync(Tp.data(), s->T, sizeof(cplx) * Tp.size(), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    if (schur_status != 0) {
        set_error("QR iteration for the Schur form of H_m did not converge");
        return SIMM_ENOCONV;
    }
    s->ritz.resize(me);
    for (int k = 0; k < me; ++k) {
        const cplx th = Tp[(size_t)k * (k + 1) / 2 + k];
        if (th.re == 0.0 && th.im == 0.0) {
            s->ritz[k] = cplx{NAN, NAN};
        } else {
            const cplx inv = cdiv(cplx{1.0, 0.0}, th);
            s->ritz[k] = cplx{s->sigma.re + inv.re, s->sigma.im + inv.im};
        }
    }
    return SIMM_OK;
}

simm_status schur_phase(simm_shift_s* s, int ldh, int* status_dev, hipStream_t st, KernelClock* clk = nullptr) {
    SIMM_TRY(schur_launch(s, ldh, status_dev, st, clk));
    return schur_finish(s, status_dev, st);
}

// y = (A - sigma B)^{-1} u with the shift's factor: the partitioned sweeps of the FP64
// factor, or those of the FP32 factor refined against the FP64 pencil.
simm_status apply_inverse(const simm_shift_s* s, const cplx* u, cplx* y, const int* active, hipStream_t st) {
    if (s->mixed) return refine_apply(s->spike, s->rpen, s->rst, u, y, active, st);
    return spike_apply(s->spike, u, y, active, st);
}

// Row blocks of the Gram-Schmidt kernels (the passes over V_j are bound by HBM: several
// workgroups per compute unit keep enough loads in flight); SIMM_GS_BLOCKS overrides.
int gs_row_blocks(int64_t n) {
    int64_t b = kGsRowBlocks;
    if (const char* e = getenv("SIMM_GS_BLOCKS")) b = std::max<int64_t>(1, atoll(e));
    return (int)std::min<int64_t>(b, std::max<int64_t>(1, (n + 63) / 64));
}

// Krylov phase of one shift (hot-path steps a3-a5) on a factored shift: the
// partitioned-sweep data of the factor (a launch wide enough to fill the device, so
// it runs here rather than beside other work), b, beta, the Arnoldi basis V_{m+1}
// and H_{m+1,m}, and the Schur data of H_m.
simm_status krylov_shift(simm_shift_s* s, const cplx* f_dev, int m, hipStream_t st, int64_t* applies,
                         KernelClock* clk = nullptr, const std::atomic<bool>* cancel = nullptr,
                         const std::function<void()>* before_schur = nullptr, bool defer_schur = false) {
    simm_pencil_s* p = s->p;
    s->m = m;
    const int64_t n = p->n;
    if (cancel && cancel->load()) {
        set_error("Krylov phase cancelled");
        return SIMM_ECANCELED;
    }
    // partitioned-sweep data (unit-state responses of every chunk), unless the
    // factor comes prepared (from another shift, or earlier on another stream)
    if (!s->factor_borrowed && !s->sweeps_ready) SIMM_TRY(prepare_sweeps(s, st, clk));
    SIMM_TRY(ensure_dev(&s->V, s->cap_V, (size_t)n * (m + 1)));
    SIMM_TRY(ensure_dev(&s->H, s->cap_H, (size_t)(m + 1) * m));
    SIMM_HIP_TRY(hipMemsetAsync(s->H, 0, sizeof(cplx) * (m + 1) * m, st));

    // scratch: Arnoldi work; flags
    const int nblk = gs_row_blocks(n);
    const int64_t rows = (n + nblk - 1) / nblk;
    const int nblk_eff = (int)((n + rows - 1) / rows);
    DevBuf work;
    const size_t bytes = sizeof(cplx) * ((size_t)nblk_eff * (m + 2) + 2 * (size_t)(m + 2) + (size_t)n) +
                         sizeof(double) * 4 + sizeof(int) * 8;
    SIMM_TRY(work.alloc(bytes + 16 * 256, st));
    char* wp = work.as<char>();
    auto take = [&](size_t b) {
        char* r = wp;
        wp += (b + 255) & ~(size_t)255;
        return r;
    };
    ArnoldiWork aw;
    aw.nblk = nblk_eff;
    aw.partial = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)nblk_eff * (m + 2)));
    aw.h1 = reinterpret_cast<cplx*>(take(sizeof(cplx) * (m + 2)));
    aw.h2 = reinterpret_cast<cplx*>(take(sizeof(cplx) * (m + 2)));
    aw.hnorm = reinterpret_cast<double*>(take(sizeof(double) * 4));
    aw.u = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)n));
    int* flags = reinterpret_cast<int*>(take(sizeof(int) * 8));   // [1] active, [2] m_eff, [3] schur status
    double* beta_d = aw.hnorm + 2;
    {
        int init[4] = {INT_MAX, 1, m, 0};
        SIMM_HIP_TRY(hipMemcpyAsync(flags, init, sizeof(init), hipMemcpyHostToDevice, st));
    }
    // the chains of this phase's applications hold their share of the device's budget
    // until the phase is done on the device
    ChainSlots slots;
    SIMM_TRY(slots.acquire(spike_chain_weight(s->spike), st));
    // a3: b = (A - sigma B)^{-1} f, beta, v_1
    {
        KScope ks(clk, SIMM_K_BAND_SWEEP);
        SIMM_TRY(apply_inverse(s, f_dev, s->V, nullptr, st));
    }
    SIMM_TRY(vec_norm_scale(n, s->V, s->V, beta_d, aw, st));
    // a4: Arnoldi steps.  With `cancel`, the host stays at most 16 steps ahead of the
    // device and stops enqueuing once *cancel is set.
    hipEvent_t ring[2] = {nullptr, nullptr};
    struct RingRelease {
        hipEvent_t* e;
        ~RingRelease() {
            for (int i = 0; i < 2; ++i)
                if (e[i]) (void)hipEventDestroy(e[i]);
        }
    } ring_release{ring};
    if (cancel)
        for (auto& e : ring) SIMM_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (int j = 0; j < m; ++j) {
        if (cancel && j % 8 == 0) {
            if (cancel->load(std::memory_order_relaxed)) {
                set_error("Krylov phase cancelled");
                return SIMM_ECANCELED;
            }
            hipEvent_t& e = ring[(j / 8) % 2];
            if (j >= 16) SIMM_HIP_TRY(hipEventSynchronize(e));
            SIMM_HIP_TRY(hipEventRecord(e, st));
        }
        cplx* vj = s->V + (int64_t)j * n;
        {
            KScope ks(clk, SIMM_K_BAND_SWEEP);   // one application of M: B v, then the factor's sweeps
            SIMM_TRY(prepare_input(n, vj, p->B, p->klb, p->kub, nullptr, flags + 1, aw.u, nullptr, st));
            SIMM_TRY(apply_inverse(s, aw.u, s->V + (int64_t)(j + 1) * n, flags + 1, st));
        }
        KScope ks(clk, SIMM_K_GRAM_SCHMIDT);
        SIMM_TRY(arnoldi_step(n, s->V, n, j, s->H, m + 1, aw, flags + 1, flags + 2, st));
    }
    int fl[4];
    int spike_err = 0, refine_err = 0;
    double beta = 0.0;
    SIMM_HIP_TRY(hipMemcpyAsync(&spike_err, s->spike.err, sizeof(int), hipMemcpyDeviceToHost, st));
    if (s->mixed) SIMM_HIP_TRY(hipMemcpyAsync(&refine_err, s->rst.flags + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipMemcpyAsync(fl, flags, sizeof(fl), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipMemcpyAsync(&beta, beta_d, sizeof(double), hipMemcpyDeviceToHost, st));
    std::vector<cplx> Hfull((size_t)(m + 1) * m);
    SIMM_HIP_TRY(hipMemcpyAsync(Hfull.data(), s->H, sizeof(cplx) * Hfull.size(), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    slots.release();
    if (spike_err != 0) {
        set_error("partitioned sweep: a chunk-chain barrier timed out");
        return SIMM_EHIP;
    }
    if (refine_err != 0) {
        char msg[200];
        std::snprintf(msg, sizeof msg, "FP32 factor at sigma = %.17g%+.17gi: iterative refinement did not reach a "
                      "backward error of %g in %d steps", s->sigma.re, s->sigma.im, kRefineTol, kRefineMaxSteps);
        set_error(msg);
        return SIMM_EREFINE;
    }
    s->m_eff = fl[2];
    s->beta = beta;
    const int me = s->m_eff;
    if (applies) *applies += me + 1;
    s->H_host.assign((size_t)(me + 1) * me, cplx{0, 0});
    for (int j = 0; j < me; ++j)
        for (int i = 0; i <= me; ++i) s->H_host[i + (size_t)j * (me + 1)] = Hfull[i + (size_t)j * (m + 1)];
    s->h_last = cabs(s->H_host[me + (size_t)(me - 1) * (me + 1)]);
    // a5: Schur form of H_m (one wavefront: the caller may start other work beside it),
    // unless the caller forms it later (from the device copy of H, leading dimension m + 1)
    if (before_schur) (*before_schur)();
    if (defer_schur) return SIMM_OK;
    SIMM_TRY(schur_phase(s, m + 1, flags + 3, st, clk));
    return SIMM_OK;
}

// The Krylov phases (steps a3-a5) of nr <= 4 spaces of one factor in lockstep: every
// application of M takes the nr current basis vectors in one pass over the factor
// (spike_apply_nr, each column as alone); the Gram-Schmidt steps, H, beta and the
// Schur forms stay per space, so each space gets exactly what krylov_shift gives it.
// kvs[r] borrow the factor (sweep data ready, FP64), and kvs[0]->spike's scratch holds
// nr columns; start vector r at F + r ldf.
simm_status krylov_block(simm_shift_s* const* kvs, int nr, const cplx* F, int64_t ldf, int m, hipStream_t st) {
    simm_shift_s* k0 = kvs[0];
    const SpikeFactor& f = k0->spike;
    if (nr < 1 || nr > 4 || nr > f.nrhs || nr > spike_max_nrhs(f) || k0->mixed) {
        set_error("Krylov spaces in lockstep: 1 to 4 FP64 spaces within the factor's scratch");
        return SIMM_EINVAL;
    }
    simm_pencil_s* p = k0->p;
    const int64_t n = p->n, n16 = f.n16;
    const int nblk = gs_row_blocks(n);
    const int64_t rows = (n + nblk - 1) / nblk;
    const int nblk_eff = (int)((n + rows - 1) / rows);
    DevBuf work[4], uy;
    ArnoldiWork aw[4];
    int* flags[4] = {};
    double* beta_d[4] = {};
    const size_t bytes = sizeof(cplx) * ((size_t)nblk_eff * (m + 2) + 2 * (size_t)(m + 2)) + sizeof(double) * 4 +
                         sizeof(int) * 8;
    for (int r = 0; r < nr; ++r) {
        simm_shift_s* s = kvs[r];
        s->m = m;
        SIMM_TRY(ensure_dev(&s->V, s->cap_V, (size_t)n * (m + 1)));
        SIMM_TRY(ensure_dev(&s->H, s->cap_H, (size_t)(m + 1) * m));
        SIMM_HIP_TRY(hipMemsetAsync(s->H, 0, sizeof(cplx) * (m + 1) * m, st));
        SIMM_TRY(work[r].alloc(bytes + 8 * 256, st));
        char* wp = work[r].as<char>();
        auto take = [&](size_t b) {
            char* q = wp;
            wp += (b + 255) & ~(size_t)255;
            return q;
        };
        aw[r].nblk = nblk_eff;
        aw[r].partial = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)nblk_eff * (m + 2)));
        aw[r].h1 = reinterpret_cast<cplx*>(take(sizeof(cplx) * (m + 2)));
        aw[r].h2 = reinterpret_cast<cplx*>(take(sizeof(cplx) * (m + 2)));
        aw[r].hnorm = reinterpret_cast<double*>(take(sizeof(double) * 4));
        aw[r].u = nullptr;   // the block's own input buffer serves every space
        flags[r] = reinterpret_cast<int*>(take(sizeof(int) * 8));   // [1] active, [2] m_eff, [3] schur status
        beta_d[r] = aw[r].hnorm + 2;
        int init[4] = {INT_MAX, 1, m, 0};
        SIMM_HIP_TRY(hipMemcpyAsync(flags[r], init, sizeof(init), hipMemcpyHostToDevice, st));
    }
    SIMM_TRY(uy.alloc(sizeof(cplx) * (size_t)n16 * nr * 2, st));
    cplx* U = uy.as<cplx>();
    cplx* Y = U + n16 * nr;
    GsBatch gb{};
    for (int r = 0; r < nr; ++r) {
        gb.V[r] = kvs[r]->V;
        gb.H[r] = kvs[r]->H;
        gb.partial[r] = aw[r].partial;
        gb.h1[r] = aw[r].h1;
        gb.h2[r] = aw[r].h2;
        gb.hnorm[r] = aw[r].hnorm;
        gb.active[r] = flags[r] + 1;
        gb.m_eff[r] = flags[r] + 2;
    }
    ChainSlots slots;
    SIMM_TRY(slots.acquire(spike_chain_weight(f), st));
    // a3: b = (A - sigma B)^{-1} f, beta, v_1
    SIMM_TRY(spike_apply_nr(f, F, ldf, Y, n16, nr, st));
    for (int r = 0; r < nr; ++r) {
        SIMM_HIP_TRY(hipMemcpyAsync(kvs[r]->V, Y + r * n16, sizeof(cplx) * n, hipMemcpyDeviceToDevice, st));
        SIMM_TRY(vec_norm_scale(n, kvs[r]->V, kvs[r]->V, beta_d[r], aw[r], st));
    }
    // a4: Arnoldi steps (a space that broke down keeps receiving applications; its
    // Gram-Schmidt steps are skipped and nothing reads those columns)
    for (int j = 0; j < m; ++j) {
        for (int r = 0; r < nr; ++r)
            SIMM_TRY(prepare_input(n, kvs[r]->V + (int64_t)j * n, p->B, p->klb, p->kub, nullptr, nullptr, U + r * n16,
                                   nullptr, st));
        SIMM_TRY(spike_apply_nr(f, U, n16, Y, n16, nr, st));
        for (int r = 0; r < nr; ++r)
            SIMM_HIP_TRY(hipMemcpyAsync(kvs[r]->V + (int64_t)(j + 1) * n, Y + r * n16, sizeof(cplx) * n,
                                        hipMemcpyDeviceToDevice, st));
        // the spaces' Gram-Schmidt steps in the same launches
        SIMM_TRY(arnoldi_step_batch(n, gb, nr, n, j, m + 1, nblk_eff, st));
    }
    int spike_err = 0;
    int fl[4][4];
    double beta[4] = {};
    std::vector<cplx> Hfull((size_t)nr * (m + 1) * m);
    SIMM_HIP_TRY(hipMemcpyAsync(&spike_err, f.err, sizeof(int), hipMemcpyDeviceToHost, st));
    for (int r = 0; r < nr; ++r) {
        SIMM_HIP_TRY(hipMemcpyAsync(fl[r], flags[r], sizeof(fl[r]), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipMemcpyAsync(&beta[r], beta_d[r], sizeof(double), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipMemcpyAsync(Hfull.data() + (size_t)r * (m + 1) * m, kvs[r]->H, sizeof(cplx) * (m + 1) * m,
                                    hipMemcpyDeviceToHost, st));
    }
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    slots.release();
    if (spike_err != 0) {
        set_error("partitioned sweep: a chunk-chain barrier timed out");
        return SIMM_EHIP;
    }
    for (int r = 0; r < nr; ++r) {
        simm_shift_s* s = kvs[r];
        s->m_eff = fl[r][2];
        s->beta = beta[r];
        const int me = s->m_eff;
        const cplx* Hr = Hfull.data() + (size_t)r * (m + 1) * m;
        s->H_host.assign((size_t)(me + 1) * me, cplx{0, 0});
        for (int j = 0; j < me; ++j)
            for (int i = 0; i <= me; ++i) s->H_host[i + (size_t)j * (me + 1)] = Hr[i + (size_t)j * (m + 1)];
        s->h_last = cabs(s->H_host[me + (size_t)(me - 1) * (me + 1)]);
    }
    // a5: the Schur forms of the nr matrices H_m side by side (each one wavefront), on st
    // and on streams of their own made for them
    struct Side {
        hipStream_t s[4] = {};
        hipEvent_t e = nullptr;
        ~Side() {
            for (auto& x : s)
                if (x) {
                    (void)hipStreamSynchronize(x);
                    (void)hipStreamDestroy(x);
                }
            if (e) (void)hipEventDestroy(e);
        }
    } side;
    SIMM_HIP_TRY(hipEventCreateWithFlags(&side.e, hipEventDisableTiming));
    SIMM_HIP_TRY(hipEventRecord(side.e, st));
    for (int r = 1; r < nr; ++r) {
        SIMM_HIP_TRY(hipStreamCreateWithFlags(&side.s[r], hipStreamNonBlocking));
        SIMM_HIP_TRY(hipStreamWaitEvent(side.s[r], side.e, 0));
    }
    auto sst = [&](int r) { return r == 0 ? st : side.s[r]; };
    for (int r = 0; r < nr; ++r) SIMM_TRY(schur_launch(kvs[r], m + 1, flags[r] + 3, sst(r)));
    for (int r = 0; r < nr; ++r) SIMM_TRY(schur_finish(kvs[r], flags[r] + 3, sst(r)));
    return SIMM_OK;
}

// Both phases of one shift (hot-path steps a1-a5).
simm_status build_shift(simm_pencil_s* p, cplx sigma, const cplx* f_dev, int m, hipStream_t st,
                        std::unique_ptr<simm_shift_s>& out, int64_t* applies, KernelClock* clk = nullptr,
                        int precision = SIMM_PREC_FP64) {
    std::unique_ptr<simm_shift_s> s;
    SIMM_TRY(factor_shift(p, sigma, st, s, clk, nullptr, precision));
    SIMM_TRY(krylov_shift(s.get(), f_dev, m, st, applies, clk));
    out = std::move(s);
    return SIMM_OK;
}

struct EvalOut {
    std::vector<double> indicator, rho, nsf, nsc, Tf;
    std::vector<uint8_t> decision;
};

// Evaluate (level, ix, iy, shift) rows on the device; results copied to host.
simm_status evaluate(const std::vector<simm_shift_s*>& shifts, const std::vector<int64_t>& regs, const simm_params* prm,
                     const Rule& rule, hipStream_t st, EvalOut& out, cplx* sums_dev, int m_sums,
                     KernelClock* clk = nullptr) {
    const int64_t N = (int64_t)regs.size() / 4;
    out.indicator.assign(N, 0);
    out.rho.assign(N, 0);
    out.nsf.assign(N, 0);
    out.nsc.assign(N, 0);
    out.Tf.assign(N, 0);
    out.decision.assign(N, 0);
    if (N == 0) return SIMM_OK;
    std::vector<ShiftDev> sd;
    int mmax = 1;
    for (auto* s : shifts) {
        sd.push_back(shift_dev(s));
        mmax = std::max(mmax, s->m_eff);
    }
    DevBuf b;
    const size_t bytes = sizeof(ShiftDev) * sd.size() + sizeof(int64_t) * regs.size() + sizeof(double) * 5 * N + N + 1024;
    SIMM_TRY(b.alloc(bytes, st));
    char* p = b.as<char>();
    ShiftDev* sdd = reinterpret_cast<ShiftDev*>(p);
    p += (sizeof(ShiftDev) * sd.size() + 255) & ~(size_t)255;
    int64_t* rd = reinterpret_cast<int64_t*>(p);
    p += (sizeof(int64_t) * regs.size() + 255) & ~(size_t)255;
    double* o = reinterpret_cast<double*>(p);
    uint8_t* dec = reinterpret_cast<uint8_t*>(o + 5 * N);
    SIMM_HIP_TRY(hipMemcpyAsync(sdd, sd.data(), sizeof(ShiftDev) * sd.size(), hipMemcpyHostToDevice, st));
    SIMM_HIP_TRY(hipMemcpyAsync(rd, regs.data(), sizeof(int64_t) * regs.size(), hipMemcpyHostToDevice, st));
    IndicatorParams ip;
    ip.x0 = prm->x0;
    ip.y0 = prm->y0;
    ip.w1 = (prm->x1 - prm->x0) / prm->n1;
    ip.eps0 = prm->eps0;
    ip.delta0 = prm->delta0;
    ip.tau = prm->tau;
    {
        KScope ks(clk, SIMM_K_INDICATORS);
        SIMM_TRY(indicators(sdd, mmax, rd, N, ip, rule.dev, o, o + N, o + 2 * N, o + 3 * N, o + 4 * N, dec, sums_dev,
                            m_sums, st));
    }
    std::vector<double> host(5 * N);
    SIMM_HIP_TRY(hipMemcpyAsync(host.data(), o, sizeof(double) * 5 * N, hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipMemcpyAsync(out.decision.data(), dec, N, hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    for (int64_t r = 0; r < N; ++r) {
        out.indicator[r] = host[r];
        out.rho[r] = host[N + r];
        out.nsf[r] = host[2 * N + r];
        out.nsc[r] = host[3 * N + r];
        out.Tf[r] = host[4 * N + r];
    }
    return SIMM_OK;
}

simm_status validate_params(const simm_params* prm, int64_t n, int* nx, int* ny, int* K) {
    if (!prm) {
        set_error("params is NULL");
        return SIMM_EINVAL;
    }
    const double vals[] = {prm->x0, prm->x1, prm->y0, prm->y1, prm->eps0, prm->delta0, prm->tau};
    for (double v : vals)
        if (!std::isfinite(v)) {
            set_error("non-finite parameter");
            return SIMM_EINVAL;
        }
    if (!(prm->x1 > prm->x0) || !(prm->y1 > prm->y0) || prm->n1 < 1) {
        set_error("empty region or n1 < 1");
        return SIMM_EINVAL;
    }
    if (prm->m < 1 || prm->m > n) {
        set_error("need 1 <= m <= n");
        return SIMM_EINVAL;
    }
    if (prm->m > 128) {
        set_error("Krylov dimension above 128 is not supported");
        return SIMM_EUNSUPPORTED;
    }
    if (prm->gauss_per_edge < 1) {
        set_error("gauss_per_edge >= 1");
        return SIMM_EINVAL;
    }
    if (prm->gauss_per_edge > 64) {
        set_error("gauss_per_edge above 64 is not supported");
        return SIMM_EUNSUPPORTED;
    }
    const double w1 = (prm->x1 - prm->x0) / prm->n1;
    const double nyf = (prm->y1 - prm->y0) / w1;
    const long long nyr = std::llround(nyf);
    if (nyr < 1 || std::fabs(nyr * w1 - (prm->y1 - prm->y0)) > 1e-12 * std::fabs(prm->y1 - prm->y0)) {
        set_error("level-1 cells must be square: (y1-y0)/((x1-x0)/n1) must be an integer");
        return SIMM_EINVAL;
    }
    *nx = prm->n1;
    *ny = (int)nyr;
    if (prm->levels > 0) {
        *K = prm->levels;
    } else {
        if (!(prm->h0 > 0) || !std::isfinite(prm->h0)) {
            set_error("h0 > 0 or levels > 0 required");
            return SIMM_EINVAL;
        }
        *K = 1 + std::max(0, (int)std::ceil(std::log2(w1 / prm->h0)));
    }
    if (*K > 60) {
        set_error("too many levels");
        return SIMM_EINVAL;
    }
    if (prm->lookahead < 0 || prm->lookahead > 16) {
        set_error("lookahead must be in 0 .. 16");
        return SIMM_EINVAL;
    }
    if (prm->precision != SIMM_PREC_FP64 && prm->precision != SIMM_PREC_MIXED) {
        set_error("precision must be SIMM_PREC_FP64 or SIMM_PREC_MIXED");
        return SIMM_EINVAL;
    }
    return SIMM_OK;
}

cplx cell_center(const simm_params* prm, int level, int64_t ix, int64_t iy) {
    const double w1 = (prm->x1 - prm->x0) / prm->n1;
    const double w = std::ldexp(w1, 1 - level);
    volatile double ax = ((double)ix + 0.5) * w;
    volatile double ay = ((double)iy + 0.5) * w;
    return cplx{prm->x0 + ax, prm->y0 + ay};
}

double cdist(cplx a, cplx b) { return std::hypot(a.re - b.re, a.im - b.im); }

std::vector<int> shift_order(const std::vector<simm_shift_s*>& shifts, cplx c, int exclude) {
    std::vector<int> idx;
    for (int s = 0; s < (int)shifts.size(); ++s)
        if (s != exclude) idx.push_back(s);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        const double da = cdist(shifts[a]->sigma, c), db = cdist(shifts[b]->sigma, c);
        if (da != db) return da < db;
        return a < b;
    });
    return idx;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st;
    double* acc;
    Timer(hipStream_t s, double* ms) : st(s), acc(ms) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, st);
    }
    ~Timer() {
        (void)hipEventRecord(b, st);
        (void)hipEventSynchronize(b);
        float t = 0;
        (void)hipEventElapsedTime(&t, a, b);
        *acc += t;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// A shift built ahead of the association order (steps 2-3), by a host thread of its
// own on a stream of its own, in phases: 0 the factor, 1 the partitioned-sweep data,
// 2 the Krylov phase.  The factor always runs; later phases run when asked for,
// before or after the earlier ones are done.  Joined (and its stream released) on
// destruction, so no thread outlives the run that started it.
struct AheadBuild {
    std::thread th;
    std::mutex mu;
    std::unique_ptr<simm_shift_s> s;
    simm_status rc = SIMM_OK;   // status of the last phase run
    std::string err;
    KernelClock clock;
    hipStream_t st = nullptr;
    std::atomic<bool> cancel{false};
    bool timed = false;
    int want = 0;        // last phase asked for
    int done = -1;       // last phase completed
    bool running = false;
    int64_t applies = 0;
    const cplx* kf = nullptr;
    int km = 0;
    hipEvent_t kready = nullptr;
    int dev = 0;
    simm_pencil_s* pen = nullptr;
    cplx sigma{0, 0};
    int precision = SIMM_PREC_FP64;

    simm_status run_phase(int ph) {
        if (ph == 0) {
            const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                st = nullptr;
                set_error(std::string("stream for a shift built ahead: ") + hipGetErrorString(e));
                return SIMM_EHIP;
            }
            clock.st = st;
            return factor_shift(pen, sigma, st, s, timed ? &clock : nullptr, &cancel, precision);
        }
        if (ph == 1) return prepare_sweeps(s.get(), st, timed ? &clock : nullptr);
        SIMM_HIP_TRY(hipStreamWaitEvent(st, kready, 0));   // f is written on the run's stream
        return krylov_shift(s.get(), kf, km, st, &applies, timed ? &clock : nullptr, &cancel);
    }
    void thread_main() {
        (void)hipSetDevice(dev);
        for (;;) {
            int ph;
            {
                std::lock_guard<std::mutex> lk(mu);
                if (rc != SIMM_OK || done >= want) {
                    running = false;
                    return;
                }
                ph = done + 1;
            }
            const simm_status r = run_phase(ph);
            std::lock_guard<std::mutex> lk(mu);
            rc = r;
            if (r != SIMM_OK) err = g_err;
            else done = ph;
        }
    }
    void start(simm_pencil_s* p, cplx sig, bool timed_, int precision_) {
        timed = timed_;
        precision = precision_;
        dev = p->dev;
        pen = p;
        sigma = sig;
        running = true;
        th = std::thread([this]() { thread_main(); });
    }
    // asks for phases up to `level` (2: the Krylov phase, start vector f written on
    // the run's stream before `ready`)
    void request(int level, const cplx* f = nullptr, int m = 0, hipEvent_t ready = nullptr) {
        bool spawn = false;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (level <= want) return;
            want = level;
            if (level >= 2) {
                kf = f;
                km = m;
                kready = ready;
            }
            if (!running && rc == SIMM_OK) running = spawn = true;
        }
        if (spawn) {   // the thread has finished what it was asked for: run the rest on a new one
            if (th.joinable()) th.join();
            th = std::thread([this]() { thread_main(); });
        }
    }
    int wanted() {
        std::lock_guard<std::mutex> lk(mu);
        return want;
    }
    // waits for the build; its kernel times go to (ms, cnt) if those are given
    void finish(double* ms = nullptr, int64_t* cnt = nullptr) {
        if (th.joinable()) th.join();
        if (ms && cnt) clock.collect(ms, cnt);
        if (st) {
            release_stream_buffers(st);   // nothing allocated in stream order outlives st
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
            st = nullptr;
        }
    }
    ~AheadBuild() { finish(); }
};

// Number of shift factors the association may compute ahead: the requested
// look-ahead (default: one per hardware queue the HIP runtime gives the process,
// GPU_MAX_HW_QUEUES, 4 unless set, less the run stream's and the side stream's, at
// most 11; more streams than queues share a queue and run one after the other), cut
// so that the factors take at most a quarter of the free device memory.
int lookahead_width(const simm_params* prm, const simm_pencil_s* p) {
    int w = prm->lookahead;
    if (w <= 0) {
        int queues = 4;
        if (const char* e = std::getenv("GPU_MAX_HW_QUEUES")) queues = std::max(1, std::atoi(e));
        w = std::min(11, std::max(1, queues - 2));
    }
    if (w <= 1) return 1;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 1;
    const int64_t n = p->n;
    const int kl = std::max(p->kla, p->klb), ku = std::max(p->kua, p->kub);
    const double per_shift = 16.0 * ((double)(2 * kl + ku + 1) * n + (double)band_lu_panel_elems(n, kl) +
                                     4.0 * (double)n * (kl + 16)) * 1.25;
    const double fit = (double)free_b / 4.0 / per_shift;
    return (int)std::max(1.0, std::min((double)w, std::floor(fit)));
}

__global__ void k_gather_sums(const cplx* sums, int m_sums, const int64_t* regs, int64_t cnt, cplx* Y) {
    // Y(:, 2q + w) = sums(:, 2 regs[q] + w)
    const int64_t col = blockIdx.x;
    if (col >= 2 * cnt) return;
    const int64_t r = regs[col / 2];
    const int w = (int)(col & 1);
    for (int i = threadIdx.x; i < m_sums; i += blockDim.x) Y[col * m_sums + i] = sums[(2 * r + w) * m_sums + i];
}

// A square of the current level and the shift it is tested with (index into the run's shifts).
struct Sq {
    int64_t ix, iy;
    int s;
};

// Frees a built shift's factor and sweep data (its Schur form and Krylov basis stay),
// after taking the refinement counters of a mixed-precision factor.
simm_status release_built_factor(simm_shift_s* sh, hipStream_t st) {
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    if (sh->mixed && sh->ref_mem) {
        unsigned long long eta_bits = 0;
        SIMM_HIP_TRY(hipMemcpyAsync(sh->saved_stats, sh->rst.stats, sizeof(sh->saved_stats), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipMemcpyAsync(&eta_bits, sh->rst.norms + 3, sizeof(eta_bits), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        std::memcpy(&sh->saved_eta, &eta_bits, sizeof(double));
    }
    sh->release_factor();
    return SIMM_OK;
}

// Steps 1-3 of the SIM-M algorithm (Sec. 3.5): the first shift at the centre of R, the
// level-1 cells and their shifts.  Leaves the shifts in R and the level-1 squares
// (cell, associated shift) in `cur`.
simm_status associate(simm_pencil_s* p, const simm_params* prm, const cplx* f_dev, hipStream_t st, simm_result_s* R,
                      const Rule& rule, KernelClock* clk, std::vector<Sq>& cur) {
    int nx, ny, K;
    SIMM_TRY(validate_params(prm, p->n, &nx, &ny, &K));
    const int m = prm->m;
    std::vector<simm_shift_s*> shifts;
    simm_status release_rc = SIMM_OK;
    auto commit = [&](std::unique_ptr<simm_shift_s> s) {
        s->borrowed = true;
        if ((prm->flags & SIMM_FLAG_RELEASE_FACTORS) && release_rc == SIMM_OK) {
            // nothing after a shift's build reads its factor (the levels need its Schur
            // form and basis only), so a run that releases its factors frees each one now
            release_rc = release_built_factor(s.get(), st);
        }
        shifts.push_back(s.get());
        R->shifts.push_back(std::move(s));
    };
    // steps 2-3 set up before step 1, so that factors for cells can start beside it:
    // the level-1 cells and their association state
    std::vector<std::pair<int64_t, int64_t>> cells;
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) cells.emplace_back(ix, iy);
    const int64_t ncell = (int64_t)cells.size();
    std::map<std::pair<int64_t, int>, bool> resolv;   // (cell, shift) -> resolvable
    // Whether a shift resolves a cell (Definition 3.1) needs only the residuals of the
    // reduced solves, which come from Hessenberg determinants of H_m (cells_resid);
    // the Schur form of each shift built on the run's stream then runs on a side
    // stream beside the next shift's work, and all of them are joined before the
    // association returns (the levels need them).
    IndicatorParams ip;
    ip.x0 = prm->x0;
    ip.y0 = prm->y0;
    ip.w1 = (prm->x1 - prm->x0) / prm->n1;
    ip.eps0 = prm->eps0;
    ip.delta0 = prm->delta0;
    ip.tau = prm->tau;
    std::vector<int64_t> cells_host;
    for (auto& c : cells) {
        cells_host.push_back(c.first);
        cells_host.push_back(c.second);
    }
    std::vector<unsigned long long> rbits_host(ncell);
    DevBuf cells_dev, rbits_dev, schur_status;
    SIMM_TRY(cells_dev.alloc(sizeof(int64_t) * cells_host.size(), st));
    SIMM_TRY(rbits_dev.alloc(sizeof(unsigned long long) * ncell, st));
    SIMM_TRY(schur_status.alloc(sizeof(int) * (ncell + 1), st));   // at most one shift per cell and the first
    SIMM_HIP_TRY(hipMemcpyAsync(cells_dev.p, cells_host.data(), sizeof(int64_t) * cells_host.size(),
                                hipMemcpyHostToDevice, st));
    // A stream of its own, made before the factors computed ahead make theirs (the HIP
    // runtime gives a new stream the hardware queue that the fewest live streams use).
    struct SideStream {   // declared after the buffers its kernels use: joined before they are freed
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        ~SideStream() {
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
            if (e) (void)hipEventDestroy(e);
        }
    } side;
    SIMM_HIP_TRY(hipStreamCreateWithFlags(&side.s, hipStreamNonBlocking));
    SIMM_HIP_TRY(hipEventCreateWithFlags(&side.e, hipEventDisableTiming));
    KernelClock side_clk;
    side_clk.st = side.s;
    std::vector<simm_shift_s*> schur_pending;   // shift k's status at schur_status[k]
    auto defer_schur = [&](simm_shift_s* sh) -> simm_status {
        SIMM_HIP_TRY(hipEventRecord(side.e, st));
        SIMM_HIP_TRY(hipStreamWaitEvent(side.s, side.e, 0));
        SIMM_TRY(schur_launch(sh, sh->m + 1, schur_status.as<int>() + schur_pending.size(), side.s,
                              clk ? &side_clk : nullptr));
        schur_pending.push_back(sh);
        return SIMM_OK;
    };
    auto eval_cells_vs = [&](int s) -> simm_status {
        Timer t(st, &R->ms[1]);
        const simm_shift_s* sh = shifts[s];
        {
            KScope ks(clk, SIMM_K_INDICATORS);
            SIMM_TRY(cells_resid(sh->H, sh->m + 1, sh->m_eff, sh->h_last, sh->sigma, cells_dev.as<int64_t>(), ncell, 1,
                                 ip, rule.dev, rbits_dev.as<unsigned long long>(), st));
        }
        SIMM_HIP_TRY(hipMemcpyAsync(rbits_host.data(), rbits_dev.p, sizeof(unsigned long long) * ncell,
                                    hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        for (int64_t c = 0; c < ncell; ++c) {
            double rho;
            std::memcpy(&rho, &rbits_host[c], sizeof rho);
            resolv[{c, s}] = rho <= prm->eps0;
        }
        return SIMM_OK;
    };
    // A cell gets a new shift (at its centre) iff no shift made so far resolves it.
    // One shift's banded LU is a chain of small launches that leaves most of the
    // device idle, so the factors of the next cells that no shift resolves yet are
    // computed ahead, concurrently on streams of their own, while the Krylov phase of
    // the current shift runs on the run's stream.  A factor made ahead is used only
    // when the cell order reaches its cell still unresolved, so the shifts kept and
    // every later result are those of the one-at-a-time order.
    const int W = lookahead_width(prm, p);
    hipEvent_t ready = nullptr;   // f is on the device (it is written on the run's stream)
    struct EventGuard {           // declared before the builds ahead: destroyed after they are joined
        hipEvent_t* e;
        ~EventGuard() {
            if (*e) (void)hipEventDestroy(*e);
        }
    } ready_guard{&ready};
    std::map<int64_t, std::unique_ptr<AheadBuild>> ahead;   // cell -> factor in flight or done
    std::vector<std::unique_ptr<AheadBuild>> dropped;         // factors whose cell got resolved
    auto release_dropped = [&]() {
        for (auto& b : dropped) b->finish(clk ? R->kms : nullptr, clk ? R->kcnt : nullptr);
        dropped.clear();
    };
    auto drop = [&](std::unique_ptr<AheadBuild> b) {
        b->cancel.store(true);
        dropped.push_back(std::move(b));
    };
    auto drop_all = [&]() {
        for (auto& kv : ahead) drop(std::move(kv.second));
        ahead.clear();
        release_dropped();
    };
    struct DropGuard {
        std::function<void()> f;
        ~DropGuard() { f(); }
    } drop_guard{drop_all};
    auto unresolved = [&](int64_t c) {
        for (int s = 0; s < (int)shifts.size(); ++s)
            if (resolv[{c, s}]) return false;
        return true;
    };
    // factors ahead for cells shift `sh` resolves will not be used
    auto drop_resolved_by = [&](int sh) {
        for (auto it = ahead.begin(); it != ahead.end();) {
            if (resolv[{it->first, sh}]) {
                drop(std::move(it->second));
                it = ahead.erase(it);
            } else {
                ++it;
            }
        }
        if ((int)dropped.size() >= W) release_dropped();   // bounds the memory they hold
    };
    // keep W factors ahead: the first cells from `from` on that no shift resolves so far
    auto top_up = [&](int64_t from) {
        if (W <= 1) return;
        int live = (int)ahead.size();
        for (int64_t d = from; d < ncell && live < W; ++d) {
            if (ahead.count(d) || !unresolved(d)) continue;
            auto b = std::make_unique<AheadBuild>();
            b->start(p, cell_center(prm, 1, cells[d].first, cells[d].second), clk != nullptr, prm->precision);
            ahead[d] = std::move(b);
            ++live;
        }
    };
    // For small factors the Krylov phases of the next KA cells predicted to need a
    // shift run ahead too, on the factor's own stream, so that one shift's Krylov
    // phase overlaps the next's.  Prediction: the first cells after the current one
    // that no shift resolves so far, skipping the current cell's neighbours while new
    // shifts have mostly resolved their neighbours so far (then a neighbour rarely
    // needs a shift of its own).  A wrong guess costs a cancelled build, never a
    // different result.  A small factor's Krylov phase is a chain of short launches
    // on a few compute units, and two of them share the device well (n = 400 band of
    // 45 KB: shift builds 450 -> 148 ms); a large one streams its factor through many
    // units per application, and beside the factors computed ahead two of them slowed
    // each other more than they overlapped (n = 40,000 band of 385 MB: ~875 -> ~950 ms
    // per step), so they stay one at a time.
    const double band_bytes =
        16.0 * (double)(2 * std::max(p->kla, p->klb) + std::max(p->kua, p->kub) + 1) * (double)p->n;
    const int KA = (W > 1 && band_bytes <= 64.0 * (1 << 20)) ? 2 : 0;
    if (KA > 0) {
        SIMM_HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
        SIMM_HIP_TRY(hipEventRecord(ready, st));
    }
    int64_t nb_hits = 0, nb_seen = 0;   // neighbours a new shift resolved / could have resolved
    auto neighbours = [&](int64_t a, int64_t b) {
        return std::llabs(cells[a].first - cells[b].first) <= 1 && std::llabs(cells[a].second - cells[b].second) <= 1;
    };
    auto request_ahead = [&](int64_t d) {
        auto it = ahead.find(d);
        if (it == ahead.end()) {
            auto b = std::make_unique<AheadBuild>();
            b->start(p, cell_center(prm, 1, cells[d].first, cells[d].second), clk != nullptr, prm->precision);
            it = ahead.emplace(d, std::move(b)).first;
        }
        it->second->request(2, f_dev, m, ready);
    };
    // Krylov phases ahead for the cells predicted after `cur` (cur = -1: before any cell)
    auto predict_ahead = [&](int64_t cur, bool guess_far_from_centre) {
        if (KA == 0) return;
        int inflight = 0;
        for (auto& kv : ahead)
            if (kv.first > cur && kv.second->wanted() >= 2) ++inflight;
        const bool skip_nb = cur >= 0 && (nb_seen == 0 || 2 * nb_hits > nb_seen);
        const cplx c0{(prm->x0 + prm->x1) / 2, (prm->y0 + prm->y1) / 2};
        const double w1 = (prm->x1 - prm->x0) / prm->n1;
        std::vector<int64_t> picked;
        for (int64_t d = cur + 1; d < ncell && inflight < KA; ++d) {
            if (!unresolved(d)) continue;
            if (guess_far_from_centre &&
                cdist(cell_center(prm, 1, cells[d].first, cells[d].second), c0) <= 1.5 * w1)
                continue;
            bool skip = skip_nb && neighbours(cur, d);
            for (int64_t q : picked) skip = skip || (skip_nb && neighbours(q, d));
            if (skip) continue;
            auto it = ahead.find(d);
            if (it != ahead.end() && it->second->wanted() >= 2) continue;
            request_ahead(d);
            picked.push_back(d);
            ++inflight;
        }
    };
    // factors for the first cells away from R's centre, ahead of the first shift's
    // own build (a guess of which cells the first shift leaves unresolved: a wrong
    // guess costs a cancelled factor, never a different result)
    if (W > 1) {
        const cplx c0{(prm->x0 + prm->x1) / 2, (prm->y0 + prm->y1) / 2};
        const double w1 = (prm->x1 - prm->x0) / prm->n1;
        for (int64_t d = 0; d < ncell && (int)ahead.size() < W; ++d) {
            const cplx cd = cell_center(prm, 1, cells[d].first, cells[d].second);
            if (cdist(cd, c0) <= 1.5 * w1) continue;
            auto b = std::make_unique<AheadBuild>();
            b->start(p, cd, clk != nullptr, prm->precision);
            ahead[d] = std::move(b);
        }
        predict_ahead(-1, true);
    }
    // A mixed-precision shift whose refined solves miss their tolerance is rebuilt with an
    // FP64 factor (the same shift, so the run's shifts and decisions do not change).
    // The Schur form is left to defer_schur.
    auto krylov_or_fp64 = [&](std::unique_ptr<simm_shift_s>& s, const std::function<void()>* before_schur) {
        simm_status rc = krylov_shift(s.get(), f_dev, m, st, &R->counters[2], clk, nullptr, before_schur, true);
        if (rc != SIMM_EREFINE) return rc;
        R->refine_fallbacks += 1;
        const cplx sig = s->sigma;
        s.reset();
        SIMM_TRY(factor_shift(p, sig, st, s, clk, nullptr, SIMM_PREC_FP64));
        return krylov_shift(s.get(), f_dev, m, st, &R->counters[2], clk, nullptr, before_schur, true);
    };
    // step 1: first shift at the centre of R
    {
        std::unique_ptr<simm_shift_s> s;
        {
            Timer t(st, &R->ms[0]);
            SIMM_TRY(factor_shift(p, cplx{(prm->x0 + prm->x1) / 2, (prm->y0 + prm->y1) / 2}, st, s, clk, nullptr,
                                  prm->precision));
            SIMM_TRY(krylov_or_fp64(s, nullptr));
            SIMM_TRY(defer_schur(s.get()));
        }
        commit(std::move(s));
    }

    SIMM_TRY(eval_cells_vs(0));
    drop_resolved_by(0);
    top_up(0);
    std::vector<int> assoc(ncell, -1);
    for (int64_t c = 0; c < ncell; ++c) {
        const cplx ctr = cell_center(prm, 1, cells[c].first, cells[c].second);
        int chosen = -1;
        for (int s : shift_order(shifts, ctr, -1))
            if (resolv[{c, s}]) {
                chosen = s;
                break;
            }
        if (chosen < 0) {
            std::unique_ptr<simm_shift_s> s;
            bool built = false;   // both phases done ahead
            bool refine_failed_ahead = false;
            if (W > 1) {
                const auto t0 = std::chrono::steady_clock::now();
                if (!ahead.count(c)) top_up(c);
                if (KA > 0) {
                    request_ahead(c);           // this cell's Krylov phase, if not asked for yet
                    predict_ahead(c, false);    // and the next cells' beside it
                }
                std::unique_ptr<AheadBuild> b = std::move(ahead[c]);
                ahead.erase(c);
                if (b) {
                    b->finish(clk ? R->kms : nullptr, clk ? R->kcnt : nullptr);
                    if (b->rc == SIMM_EREFINE) refine_failed_ahead = true;
                    if (b->rc == SIMM_OK && b->done >= 2) {
                        s = std::move(b->s);
                        R->counters[2] += b->applies;
                        built = true;
                    } else if (b->rc == SIMM_OK && b->done >= 0) {
                        s = std::move(b->s);   // factor (and maybe sweep data) only
                    }
                }
                R->ms[0] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            }
            if (!s) {
                // one at a time (also after a failed build ahead, whose error the
                // one-at-a-time order then reports itself)
                drop_all();
                Timer t(st, &R->ms[0]);
                if (refine_failed_ahead) R->refine_fallbacks += 1;
                SIMM_TRY(factor_shift(p, ctr, st, s, clk, nullptr, refine_failed_ahead ? SIMM_PREC_FP64 : prm->precision));
            }
            if (!built) {
                // while this shift's Schur form runs (one wavefront), the sweep data of
                // the cell predicted to need a shift next is prepared on its stream
                const std::function<void()> prep_next = [&]() {
                    if (W <= 1) return;
                    const bool skip_nb = nb_seen == 0 || 2 * nb_hits > nb_seen;
                    for (int64_t d = c + 1; d < ncell; ++d) {
                        if (!unresolved(d) || (skip_nb && neighbours(c, d))) continue;
                        auto it = ahead.find(d);
                        if (it != ahead.end()) it->second->request(1);
                        break;
                    }
                };
                Timer t(st, &R->ms[0]);
                SIMM_TRY(krylov_or_fp64(s, &prep_next));
                SIMM_TRY(defer_schur(s.get()));
            }
            // neighbours of c after it that no shift resolved before this one
            std::vector<int64_t> nb;
            for (int64_t d = c + 1; d < ncell; ++d)
                if (neighbours(c, d) && unresolved(d)) nb.push_back(d);
            commit(std::move(s));
            chosen = (int)shifts.size() - 1;
            SIMM_TRY(eval_cells_vs(chosen));
            for (int64_t d : nb) nb_hits += resolv[{d, chosen}] ? 1 : 0;
            nb_seen += (int64_t)nb.size();
            drop_resolved_by(chosen);
            top_up(c + 1);
        }
        assoc[c] = chosen;
    }
    drop_all();
    SIMM_TRY(release_rc);
    {
        Timer t(st, &R->ms[0]);
        for (size_t k = 0; k < schur_pending.size(); ++k)
            SIMM_TRY(schur_finish(schur_pending[k], schur_status.as<int>() + k, side.s));
    }
    if (clk) side_clk.collect(R->kms, R->kcnt);
    cur.clear();
    for (int64_t c = 0; c < ncell; ++c) cur.push_back({cells[c].first, cells[c].second, assoc[c]});
    return SIMM_OK;
}

// Steps 4-5 (Sec. 3.5): the levels of one pencil from its level-1 squares; every
// square keeps its parent's shift unless that one does not resolve it (then the other
// shifts nearest-first), and marked squares are split into four.
simm_status level_loop(simm_pencil_s* p, const simm_params* prm, hipStream_t st, simm_result_s* R, const Rule& rule,
                       KernelClock* clk, std::vector<Sq> cur) {
    const int K = R->K;
    const int m = prm->m;
    const bool do_proj = (prm->flags & SIMM_FLAG_PROJECT) != 0;
    const int64_t maxreg = prm->max_regions_per_level > 0 ? prm->max_regions_per_level : ((int64_t)1 << 22);
    std::vector<simm_shift_s*> shifts;
    for (auto& sh : R->shifts) shifts.push_back(sh.get());
    const int m_sums = m;
    DevBuf sums_buf, sums_fb, Ybuf, nrm_buf, scr_buf, idx_buf;
    const int64_t n = p->n;
    for (int k = 1; k <= K; ++k) {
        const int64_t N = (int64_t)cur.size();
        if (N > maxreg) {
            char msg[128];
            std::snprintf(msg, sizeof msg, "level %d holds %lld squares (limit %lld)", k, (long long)N,
                          (long long)maxreg);
            set_error(msg);
            return SIMM_ELIMIT;
        }
        std::vector<int64_t> regs;
        regs.reserve(4 * N);
        for (auto& q : cur) {
            regs.push_back(k);
            regs.push_back(q.ix);
            regs.push_back(q.iy);
            regs.push_back(q.s);
        }
        cplx* sums_dev = nullptr;
        if (do_proj) {
            SIMM_TRY(sums_buf.alloc(sizeof(cplx) * (size_t)N * 2 * m_sums, st));
            sums_dev = sums_buf.as<cplx>();
        }
        EvalOut eo;
        {
            Timer t(st, &R->ms[1]);
            SIMM_TRY(evaluate(shifts, regs, prm, rule, st, eo, sums_dev, m_sums, clk));
        }
        std::vector<int> used(N);
        for (int64_t r = 0; r < N; ++r) used[r] = cur[r].s;
        // fallback: other shifts nearest-first for squares the inherited shift does not resolve
        std::vector<int64_t> pend;
        for (int64_t r = 0; r < N; ++r)
            if (eo.decision[r] == SIMM_UNRESOLVED) pend.push_back(r);
        std::map<int64_t, std::vector<int>> cand;
        for (int64_t r : pend) cand[r] = shift_order(shifts, cell_center(prm, k, cur[r].ix, cur[r].iy), cur[r].s);
        // rounds of 1, 2, 4, ... candidates per square (each round one launch): a square
        // takes the first of its candidates, in nearest-first order, that resolves it, so
        // the outcome is that of trying them one at a time
        for (size_t lo = 0, width = 1; !pend.empty(); lo += width, width *= 2) {
            std::vector<int64_t> tryr, tregs;   // tryr: square of each row
            std::vector<size_t> gbeg;           // first row of each pending square's group
            for (int64_t r : pend) {
                gbeg.push_back(tryr.size());
                const auto& cr = cand[r];
                for (size_t c = lo; c < std::min(cr.size(), lo + width); ++c) {
                    tryr.push_back(r);
                    tregs.insert(tregs.end(), {(int64_t)k, cur[r].ix, cur[r].iy, (int64_t)cr[c]});
                }
            }
            gbeg.push_back(tryr.size());
            if (tryr.empty()) break;
            cplx* fb_dev = nullptr;
            if (do_proj) {
                SIMM_TRY(sums_fb.alloc(sizeof(cplx) * tryr.size() * 2 * m_sums, st));
                fb_dev = sums_fb.as<cplx>();
            }
            EvalOut e2;
            {
                Timer t(st, &R->ms[1]);
                SIMM_TRY(evaluate(shifts, tregs, prm, rule, st, e2, fb_dev, m_sums, clk));
            }
            std::vector<int64_t> still;
            for (size_t g = 0; g + 1 < gbeg.size(); ++g) {
                const int64_t r = pend[g];
                size_t hit = gbeg[g + 1];
                for (size_t q = gbeg[g]; q < gbeg[g + 1]; ++q)
                    if (e2.decision[q] != SIMM_UNRESOLVED) {
                        hit = q;
                        break;
                    }
                if (hit < gbeg[g + 1]) {
                    const size_t q = hit;
                    eo.indicator[r] = e2.indicator[q];
                    eo.rho[r] = e2.rho[q];
                    eo.nsf[r] = e2.nsf[q];
                    eo.nsc[r] = e2.nsc[q];
                    eo.Tf[r] = e2.Tf[q];
                    eo.decision[r] = e2.decision[q];
                    used[r] = (int)tregs[4 * q + 3];
                    if (do_proj)
                        SIMM_HIP_TRY(hipMemcpyAsync(sums_dev + (size_t)r * 2 * m_sums, fb_dev + q * 2 * m_sums,
                                                    sizeof(cplx) * 2 * m_sums, hipMemcpyDeviceToDevice, st));
                } else if (gbeg[g + 1] > gbeg[g]) {
                    still.push_back(r);   // candidates left to try
                }
            }
            pend.swap(still);
        }
        R->counters[0] += N * 12 * (int64_t)prm->gauss_per_edge;
        R->counters[1] += N;
        LevelRec L;
        L.ix.resize(N);
        L.iy.resize(N);
        L.shift.resize(N);
        L.full_indicator.assign(N, NAN);
        for (int64_t r = 0; r < N; ++r) {
            L.ix[r] = cur[r].ix;
            L.iy[r] = cur[r].iy;
            L.shift[r] = used[r];
        }
        L.indicator = eo.indicator;
        L.rho_max = eo.rho;
        L.nsf = eo.nsf;
        L.nsc = eo.nsc;
        L.Tf = eo.Tf;
        L.decision = eo.decision;

        // a9: X = V_m Y for the squares of this level, shift by shift
        if (do_proj) {
            Timer t(st, &R->ms[2]);
            const bool mixed_proj = (prm->flags & SIMM_FLAG_MIXED_PROJECT) || prm->precision == SIMM_PREC_MIXED;
            const int proj_prec = !mixed_proj ? SIMM_PROJ_FP64 : (k <= 2) ? SIMM_PROJ_BF16 : SIMM_PROJ_FP32;
            std::vector<std::vector<int64_t>> by_shift(shifts.size());
            for (int64_t r = 0; r < N; ++r) by_shift[used[r]].push_back(r);
            int64_t cmax = 0;
            for (auto& v : by_shift) cmax = std::max<int64_t>(cmax, 2 * (int64_t)v.size());
            SIMM_TRY(Ybuf.alloc(sizeof(cplx) * (size_t)cmax * m_sums, st));
            SIMM_TRY(nrm_buf.alloc(sizeof(double) * (size_t)cmax, st));
            SIMM_TRY(scr_buf.alloc(sizeof(double) * (size_t)project_scratch_elems(n, cmax), st));
            SIMM_TRY(idx_buf.alloc(sizeof(int64_t) * (size_t)std::max<int64_t>(1, N), st));
            std::vector<double> nrm_host;
            for (size_t s = 0; s < shifts.size(); ++s) {
                const auto& rs = by_shift[s];
                if (rs.empty()) continue;
                const int64_t cnt = (int64_t)rs.size();
                SIMM_HIP_TRY(hipMemcpyAsync(idx_buf.p, rs.data(), sizeof(int64_t) * cnt, hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_gather_sums, dim3((unsigned)(2 * cnt)), dim3(128), 0, st, (const cplx*)sums_dev,
                                   m_sums, idx_buf.as<const int64_t>(), cnt, Ybuf.as<cplx>());
                SIMM_HIP_TRY(hipGetLastError());
                {
                    KScope ks(clk, SIMM_K_PROJECT);
                    // only the column norms are needed: X itself is not written
                    SIMM_TRY(project(n, shifts[s]->m_eff, shifts[s]->V, n, Ybuf.as<const cplx>(), m_sums, 2 * cnt,
                                     nullptr, nrm_buf.as<double>(), scr_buf.as<double>(),
                                     project_scratch_elems(n, cmax), proj_prec, st));
                }
                nrm_host.assign(2 * cnt, 0.0);
                SIMM_HIP_TRY(hipMemcpyAsync(nrm_host.data(), nrm_buf.p, sizeof(double) * 2 * cnt,
                                            hipMemcpyDeviceToHost, st));
                SIMM_HIP_TRY(hipStreamSynchronize(st));
                for (int64_t q = 0; q < cnt; ++q) L.full_indicator[rs[q]] = nrm_host[2 * q + 1] / nrm_host[2 * q];
            }
        }
        R->levels.push_back(std::move(L));
        if (k < K) {
            std::vector<Sq> nxt;
            for (int64_t r = 0; r < N; ++r) {
                if (eo.decision[r] == SIMM_REJECTED) continue;
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) nxt.push_back({2 * cur[r].ix + a, 2 * cur[r].iy + b, used[r]});
            }
            std::stable_sort(nxt.begin(), nxt.end(), [](const Sq& u, const Sq& v) {
                if (u.iy != v.iy) return u.iy < v.iy;
                return u.ix < v.ix;
            });
            cur.swap(nxt);
        }
    }

    return SIMM_OK;
}

// Steps 6-7 (Sec. 3.5): the marked level-K squares merged into 8-connected clusters.
void make_clusters(simm_result_s* R) {
    const simm_params* prm = &R->prm;
    const int K = R->K;
    const LevelRec& last = R->levels.back();
    std::map<std::pair<int64_t, int64_t>, int64_t> pos;
    std::vector<int64_t> marked;
    for (int64_t r = 0; r < (int64_t)last.decision.size(); ++r)
        if (last.decision[r] != SIMM_REJECTED) {
            marked.push_back(r);
            pos[{last.ix[r], last.iy[r]}] = r;
        }
    std::set<std::pair<int64_t, int64_t>> seen;
    const double wK = std::ldexp((prm->x1 - prm->x0) / prm->n1, 1 - K);
    for (int64_t r0 : marked) {
        const std::pair<int64_t, int64_t> key{last.ix[r0], last.iy[r0]};
        if (seen.count(key)) continue;
        std::vector<int64_t> comp;
        std::vector<std::pair<int64_t, int64_t>> stack{key};
        seen.insert(key);
        while (!stack.empty()) {
            auto cu = stack.back();
            stack.pop_back();
            comp.push_back(pos[cu]);
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    std::pair<int64_t, int64_t> nb{cu.first + dx, cu.second + dy};
                    if (pos.count(nb) && !seen.count(nb)) {
                        seen.insert(nb);
                        stack.push_back(nb);
                    }
                }
        }
        std::sort(comp.begin(), comp.end(), [&](int64_t a, int64_t b) {
            if (last.iy[a] != last.iy[b]) return last.iy[a] < last.iy[b];
            return last.ix[a] < last.ix[b];
        });
        double sr = 0, si = 0, xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
        int flags = 0;
        for (int64_t q : comp) {
            const cplx c = cell_center(prm, K, last.ix[q], last.iy[q]);
            sr += c.re;
            si += c.im;
            xmin = std::min(xmin, c.re);
            xmax = std::max(xmax, c.re);
            ymin = std::min(ymin, c.im);
            ymax = std::max(ymax, c.im);
            if (last.decision[q] == SIMM_UNRESOLVED) flags |= 1;
        }
        ClusterRec cr;
        cr.members = comp;
        cr.lam = cplx{sr / comp.size(), si / comp.size()};
        cr.shift = last.shift[comp[0]];
        cr.flags = flags;
        cr.lam_ritz = cplx{NAN, NAN};
        double best = INFINITY;
        for (const cplx& rv : R->shifts[cr.shift]->ritz) {
            if (!std::isfinite(rv.re) || !std::isfinite(rv.im)) continue;
            if (rv.re < xmin - wK || rv.re > xmax + wK || rv.im < ymin - wK || rv.im > ymax + wK) continue;
            const double d = cdist(rv, cr.lam);
            if (d < best) {
                best = d;
                cr.lam_ritz = rv;
            }
        }
        R->clusters.push_back(cr);
    }
}

// Refinement counters of the mixed-precision shifts, then the large per-shift data freed
// if asked for.
simm_status finish_run(simm_result_s* R, hipStream_t st) {
    const simm_params* prm = &R->prm;
    for (auto& sh : R->shifts) {
        if (!sh->mixed) continue;
        if (sh->mixed_stats_saved) {
            R->refine_solves += sh->saved_stats[0];
            R->refine_corrections += sh->saved_stats[1];
            R->refine_max_eta = std::max(R->refine_max_eta, sh->saved_eta);
            continue;
        }
        long long stats[2] = {0, 0};
        unsigned long long eta_bits = 0;
        SIMM_HIP_TRY(hipMemcpyAsync(stats, sh->rst.stats, sizeof(stats), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipMemcpyAsync(&eta_bits, sh->rst.norms + 3, sizeof(eta_bits), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        double eta = 0.0;
        std::memcpy(&eta, &eta_bits, sizeof(eta));
        R->refine_solves += stats[0];
        R->refine_corrections += stats[1];
        R->refine_max_eta = std::max(R->refine_max_eta, eta);
    }
    if (prm->flags & SIMM_FLAG_RELEASE_FACTORS) {
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        for (auto& sh : R->shifts) sh->release_large();
    }
    return SIMM_OK;
}

simm_status run(simm_pencil_s* p, const simm_params* prm, const cplx* f_dev, hipStream_t st, simm_result_s* R) {
    int nx, ny, K;
    SIMM_TRY(validate_params(prm, p->n, &nx, &ny, &K));
    R->K = K;
    R->prm = *prm;
    R->pencil = p;
    Rule rule;
    SIMM_TRY(rule.make(prm->gauss_per_edge, st));
    KernelClock clock;
    clock.st = st;
    KernelClock* clk = (prm->flags & SIMM_FLAG_KERNEL_TIMING) ? &clock : nullptr;
    struct Collect {
        KernelClock* c;
        simm_result_s* R;
        ~Collect() {
            if (c) c->collect(R->kms, R->kcnt);
        }
    } collect_at_exit{clk, R};
    std::vector<Sq> cur;
    SIMM_TRY(associate(p, prm, f_dev, st, R, rule, clk, cur));
    SIMM_TRY(level_loop(p, prm, st, R, rule, clk, std::move(cur)));
    make_clusters(R);
    return finish_run(R, st);
}

// ---------------------------------------------------------------------------
// Batched form, level by level (Sec. 3.3: all squares of a level are evaluated
// together): every pencil's shifts are built first (steps 1-3, pencils in flight on
// streams of their own); then each level of all pencils is one persistent indicator
// launch and one grouped projection, each a captured graph replayed per level.
// ---------------------------------------------------------------------------

// Launch shapes picked by timed replays of the captured graphs, per shape class
// (a process-wide cache: the candidates give identical results, only the time differs).
struct Autotune {
    std::mutex mu;
    std::map<std::tuple<int, int, int>, int> ind;    // (m, g, log2 rows) -> workgroups
    std::map<std::tuple<int, int>, int> proj;        // (m, log2 tiles) -> workgroups
    int64_t trials = 0;
};
Autotune g_tune;

int log2_bucket(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x && b < 62) ++b;
    return b;
}

// host-side table of a graph-captured stream segment
struct Graph {
    hipGraphExec_t exec = nullptr;
    ~Graph() { reset(); }
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
    simm_status capture(hipStream_t st, const std::function<simm_status()>& body) {
        reset();
        hipGraph_t g = nullptr;
        SIMM_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const simm_status rc = body();
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (rc != SIMM_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            return SIMM_EHIP;
        }
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            exec = nullptr;
            set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
            return SIMM_EHIP;
        }
        return SIMM_OK;
    }
    simm_status launch(hipStream_t st) {
        SIMM_HIP_TRY(hipGraphLaunch(exec, st));
        return SIMM_OK;
    }
};

struct GatherDesc {           // Y(:, col) = sums(:, src[col]) for col < ncols[0]
    const cplx* sums;
    int64_t m_sums;
    const int64_t* src;
    const int64_t* ncols;
    cplx* Y;
};

__global__ void k_gather_cols(const GatherDesc* __restrict__ dp) {
    const GatherDesc d = *dp;
    const int64_t nc = *d.ncols;
    for (int64_t col = blockIdx.x; col < nc; col += gridDim.x) {
        const int64_t s = d.src[col];
        for (int i = threadIdx.x; i < d.m_sums; i += blockDim.x) d.Y[col * d.m_sums + i] = d.sums[s * d.m_sums + i];
    }
}

// The evaluation of a list of rows (level, ix, iy, global shift, pencil) in persistent
// launches, with buffers that grow by doubling; the graph is captured again when they do
// (its kernel arguments point at them) and once per tuned launch shape.
struct IndEval {
    const ShiftDev* shifts = nullptr;
    const IndicatorParams* geo = nullptr;
    RuleDev rule{};
    int mmax = 1, m_sums = 1, g = 1;
    int64_t cap = 0;
    void* mem = nullptr;              // rows, count, outputs, sums
    int64_t* rows = nullptr;
    int64_t* nrows = nullptr;
    double* out = nullptr;            // 5 x cap
    uint8_t* dec = nullptr;
    cplx* sums = nullptr;             // cap x 2 x m_sums
    Graph graph;
    int grid = 0;                     // launch shape of the captured graph
    ~IndEval() { (void)hipFree(mem); }
    simm_status ensure(int64_t N) {
        if (N <= cap) return SIMM_OK;
        int64_t c = std::max<int64_t>(cap, 1024);
        while (c < N) c *= 2;
        (void)hipFree(mem);
        mem = nullptr;
        graph.reset();
        grid = 0;
        const size_t bytes = sizeof(int64_t) * (size_t)(5 * c + 64) + sizeof(double) * 5 * (size_t)c + (size_t)c + 256 +
                             sizeof(cplx) * (size_t)c * 2 * m_sums + 1024;
        SIMM_HIP_TRY(hipMalloc(&mem, bytes));
        char* p = reinterpret_cast<char*>(mem);
        auto take = [&](size_t b) {
            char* r = p;
            p += (b + 255) & ~(size_t)255;
            return r;
        };
        rows = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * 5 * (size_t)c));
        nrows = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * 8));
        out = reinterpret_cast<double*>(take(sizeof(double) * 5 * (size_t)c));
        dec = reinterpret_cast<uint8_t*>(take((size_t)c));
        sums = reinterpret_cast<cplx*>(take(sizeof(cplx) * (size_t)c * 2 * m_sums));
        cap = c;
        return SIMM_OK;
    }
    simm_status capture(int G, hipStream_t st) {
        grid = G;
        return graph.capture(st, [&]() {
            return indicators_persist(shifts, mmax, rows, nrows, geo, rule, G, out, out + cap, out + 2 * cap,
                                      out + 3 * cap, out + 4 * cap, dec, sums, m_sums, st);
        });
    }
    // evaluates rows[0 .. N) (host rows, 5 per square); results in host vectors
    simm_status run(const std::vector<int64_t>& hrows, hipStream_t st, EvalOut& eo) {
        const int64_t N = (int64_t)hrows.size() / 5;
        eo.indicator.assign(N, 0);
        eo.rho.assign(N, 0);
        eo.nsf.assign(N, 0);
        eo.nsc.assign(N, 0);
        eo.Tf.assign(N, 0);
        eo.decision.assign(N, 0);
        if (N == 0) return SIMM_OK;
        SIMM_TRY(ensure(N));
        SIMM_HIP_TRY(hipMemcpyAsync(rows, hrows.data(), sizeof(int64_t) * hrows.size(), hipMemcpyHostToDevice, st));
        SIMM_HIP_TRY(hipMemcpyAsync(nrows, &N, sizeof(int64_t), hipMemcpyHostToDevice, st));
        // launch shape: cached per (m, g, log2 N), else the fastest of a few timed replays
        const auto key = std::make_tuple(mmax, g, log2_bucket(N));
        int G = 0;
        {
            std::lock_guard<std::mutex> lk(g_tune.mu);
            auto it = g_tune.ind.find(key);
            if (it != g_tune.ind.end()) G = it->second;
        }
        if (G == 0) {
            float best = 1e30f;
            for (int cand : {256, 512, 1024, 2048}) {
                if (cand > 4 * N && cand > 256) break;
                SIMM_TRY(capture(cand, st));
                hipEvent_t a, b;
                SIMM_HIP_TRY(hipEventCreate(&a));
                SIMM_HIP_TRY(hipEventCreate(&b));
                SIMM_HIP_TRY(hipEventRecord(a, st));
                SIMM_TRY(graph.launch(st));
                SIMM_HIP_TRY(hipEventRecord(b, st));
                SIMM_HIP_TRY(hipEventSynchronize(b));
                float ms = 0;
                (void)hipEventElapsedTime(&ms, a, b);
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                if (ms < best) {
                    best = ms;
                    G = cand;
                }
            }
            std::lock_guard<std::mutex> lk(g_tune.mu);
            g_tune.ind[key] = G;
            g_tune.trials += 1;
        }
        if (grid != G || !graph.exec) SIMM_TRY(capture(G, st));
        SIMM_TRY(graph.launch(st));
        std::vector<double> host(5 * (size_t)cap);
        for (int q = 0; q < 5; ++q)
            SIMM_HIP_TRY(hipMemcpyAsync(host.data() + (size_t)q * N, out + (size_t)q * cap, sizeof(double) * N,
                                        hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipMemcpyAsync(eo.decision.data(), dec, N, hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        for (int64_t r = 0; r < N; ++r) {
            eo.indicator[r] = host[r];
            eo.rho[r] = host[N + r];
            eo.nsf[r] = host[2 * N + r];
            eo.nsc[r] = host[3 * N + r];
            eo.Tf[r] = host[4 * N + r];
        }
        return SIMM_OK;
    }
};

// Grouped projection of a level: gather of the sums into Y, X_g = V_g Y_g column norms
// for every (pencil, shift) group, as one captured graph over device tables.
struct ProjEval {
    void* tab = nullptr;              // GatherDesc, counts, ProjGroup table
    GatherDesc* desc = nullptr;
    int64_t* counts = nullptr;        // [0] columns, [1] groups
    ProjGroup* groups = nullptr;
    int64_t gcap = 0;
    DevBuf src, Y, scr, norms;
    Graph graph;
    int grid = 0, gz = 0;
    ~ProjEval() { (void)hipFree(tab); }
    simm_status capture(int G, hipStream_t st) {
        grid = G;
        gz = (int)std::min<int64_t>(gcap, 64);
        return graph.capture(st, [&]() {
            hipLaunchKernelGGL(k_gather_cols, dim3(1024), dim3(128), 0, st, (const GatherDesc*)desc);
            SIMM_HIP_TRY(hipGetLastError());
            return project_groups(groups, counts + 1, G, gz, st);
        });
    }
};

// One pencil of a batch between the phases.
struct BatchItem {
    simm_pencil_s* p = nullptr;
    simm_params prm{};
    std::unique_ptr<simm_result_s> R;
    std::vector<Sq> cur;
    simm_status rc = SIMM_OK;
    std::string msg;
    int64_t soff = 0;                 // first global shift index
};

// progress lines on stderr (SIMM_BATCH_PROGRESS=1): long batches otherwise print nothing
bool batch_progress() {
    static const bool on = [] {
        const char* e = std::getenv("SIMM_BATCH_PROGRESS");
        return e && e[0] == '1';
    }();
    return on;
}

simm_status run_batch_levels(std::vector<BatchItem>& items, hipStream_t st) {
    const int nb = (int)items.size();
    if (nb == 0) return SIMM_OK;
    const simm_params& p0 = items[0].prm;
    const int m = p0.m, g = p0.gauss_per_edge;
    // global shift table and per-pencil geometry
    std::vector<ShiftDev> sd;
    std::vector<IndicatorParams> geo;
    int mmax = 1, Kmax = 0;
    for (auto& it : items) {
        it.soff = (int64_t)sd.size();
        for (auto& sh : it.R->shifts) {
            sd.push_back(shift_dev(sh.get()));
            mmax = std::max(mmax, sh->m_eff);
        }
        IndicatorParams ip;
        ip.x0 = it.prm.x0;
        ip.y0 = it.prm.y0;
        ip.w1 = (it.prm.x1 - it.prm.x0) / it.prm.n1;
        ip.eps0 = it.prm.eps0;
        ip.delta0 = it.prm.delta0;
        ip.tau = it.prm.tau;
        geo.push_back(ip);
        Kmax = std::max(Kmax, it.R->K);
    }
    DevBuf tables;
    const size_t sd_bytes = (sizeof(ShiftDev) * sd.size() + 255) & ~(size_t)255;
    SIMM_TRY(tables.alloc(sd_bytes + sizeof(IndicatorParams) * geo.size() + 256, st));
    ShiftDev* sdd = tables.as<ShiftDev>();
    IndicatorParams* geod = reinterpret_cast<IndicatorParams*>(tables.as<char>() + sd_bytes);
    SIMM_HIP_TRY(hipMemcpyAsync(sdd, sd.data(), sizeof(ShiftDev) * sd.size(), hipMemcpyHostToDevice, st));
    SIMM_HIP_TRY(hipMemcpyAsync(geod, geo.data(), sizeof(IndicatorParams) * geo.size(), hipMemcpyHostToDevice, st));
    Rule rule;
    SIMM_TRY(rule.make(g, st));
    IndEval main_eval, fb_eval;
    for (IndEval* e : {&main_eval, &fb_eval}) {
        e->shifts = sdd;
        e->geo = geod;
        e->rule = rule.dev;
        e->mmax = mmax;
        e->m_sums = m;
        e->g = g;
    }
    ProjEval pe;
    const bool do_proj = (p0.flags & SIMM_FLAG_PROJECT) != 0;
    const bool mixed_proj = (p0.flags & SIMM_FLAG_MIXED_PROJECT) || p0.precision == SIMM_PREC_MIXED;
    for (int k = 1; k <= Kmax; ++k) {
        // rows of every pencil that has this level, pencil by pencil
        std::vector<int64_t> rows, first(nb + 1, 0);
        for (int i = 0; i < nb; ++i) {
            auto& it = items[i];
            first[i] = (int64_t)rows.size() / 5;
            if (k > it.R->K) continue;
            const int64_t maxreg =
                it.prm.max_regions_per_level > 0 ? it.prm.max_regions_per_level : ((int64_t)1 << 22);
            if ((int64_t)it.cur.size() > maxreg) {
                char msg[128];
                std::snprintf(msg, sizeof msg, "pencil %d: level %d holds %lld squares (limit %lld)", i, k,
                              (long long)it.cur.size(), (long long)maxreg);
                set_error(msg);
                return SIMM_ELIMIT;
            }
            for (auto& q : it.cur) rows.insert(rows.end(), {(int64_t)k, q.ix, q.iy, it.soff + q.s, (int64_t)i});
        }
        first[nb] = (int64_t)rows.size() / 5;
        const int64_t N = first[nb];
        if (batch_progress()) std::fprintf(stderr, "[simm batch] level %d: %lld squares\n", k, (long long)N);
        EvalOut eo;
        SIMM_TRY(main_eval.run(rows, st, eo));
        std::vector<int> used((size_t)N);
        for (int i = 0; i < nb; ++i)
            for (int64_t r = first[i]; r < first[i + 1]; ++r) used[r] = items[i].cur[r - first[i]].s;
        // fallback: other shifts of the same pencil nearest-first, all pencils' rounds together
        std::vector<int64_t> pend;
        std::map<int64_t, std::vector<int>> cand;
        for (int i = 0; i < nb; ++i) {
            auto& it = items[i];
            std::vector<simm_shift_s*> shv;
            for (auto& sh : it.R->shifts) shv.push_back(sh.get());
            for (int64_t r = first[i]; r < first[i + 1]; ++r)
                if (eo.decision[r] == SIMM_UNRESOLVED) {
                    pend.push_back(r);
                    const Sq& q = it.cur[r - first[i]];
                    cand[r] = shift_order(shv, cell_center(&it.prm, k, q.ix, q.iy), q.s);
                }
        }
        auto pencil_of = [&](int64_t r) {
            return (int)(std::upper_bound(first.begin(), first.end(), r) - first.begin()) - 1;
        };
        // rounds of 1, 2, 4, ... candidates per square, as in the single-pencil loop
        for (size_t lo = 0, width = 1; !pend.empty(); lo += width, width *= 2) {
            std::vector<int64_t> tryr, trows;
            std::vector<size_t> gbeg;
            for (int64_t r : pend) {
                gbeg.push_back(tryr.size());
                const auto& cr = cand[r];
                const int i = pencil_of(r);
                for (size_t c = lo; c < std::min(cr.size(), lo + width); ++c) {
                    tryr.push_back(r);
                    trows.insert(trows.end(), {(int64_t)k, rows[5 * r + 1], rows[5 * r + 2],
                                               items[i].soff + cr[c], (int64_t)i});
                }
            }
            gbeg.push_back(tryr.size());
            if (tryr.empty()) break;
            EvalOut e2;
            SIMM_TRY(fb_eval.run(trows, st, e2));
            std::vector<int64_t> still;
            for (size_t g = 0; g + 1 < gbeg.size(); ++g) {
                const int64_t r = pend[g];
                size_t hit = gbeg[g + 1];
                for (size_t q = gbeg[g]; q < gbeg[g + 1]; ++q)
                    if (e2.decision[q] != SIMM_UNRESOLVED) {
                        hit = q;
                        break;
                    }
                if (hit < gbeg[g + 1]) {
                    const size_t q = hit;
                    eo.indicator[r] = e2.indicator[q];
                    eo.rho[r] = e2.rho[q];
                    eo.nsf[r] = e2.nsf[q];
                    eo.nsc[r] = e2.nsc[q];
                    eo.Tf[r] = e2.Tf[q];
                    eo.decision[r] = e2.decision[q];
                    used[r] = (int)(trows[5 * q + 3] - items[pencil_of(r)].soff);
                    if (do_proj)
                        SIMM_HIP_TRY(hipMemcpyAsync(main_eval.sums + (size_t)r * 2 * m, fb_eval.sums + q * 2 * m,
                                                    sizeof(cplx) * 2 * m, hipMemcpyDeviceToDevice, st));
                } else if (gbeg[g + 1] > gbeg[g]) {
                    still.push_back(r);
                }
            }
            pend.swap(still);
        }
        // level records
        for (int i = 0; i < nb; ++i) {
            auto& it = items[i];
            if (k > it.R->K) continue;
            const int64_t n0 = first[i], Ni = first[i + 1] - n0;
            it.R->counters[0] += Ni * 12 * (int64_t)it.prm.gauss_per_edge;
            it.R->counters[1] += Ni;
            LevelRec L;
            L.ix.resize(Ni);
            L.iy.resize(Ni);
            L.shift.resize(Ni);
            L.full_indicator.assign(Ni, NAN);
            for (int64_t r = 0; r < Ni; ++r) {
                L.ix[r] = it.cur[r].ix;
                L.iy[r] = it.cur[r].iy;
                L.shift[r] = used[n0 + r];
            }
            L.indicator.assign(eo.indicator.begin() + n0, eo.indicator.begin() + n0 + Ni);
            L.rho_max.assign(eo.rho.begin() + n0, eo.rho.begin() + n0 + Ni);
            L.nsf.assign(eo.nsf.begin() + n0, eo.nsf.begin() + n0 + Ni);
            L.nsc.assign(eo.nsc.begin() + n0, eo.nsc.begin() + n0 + Ni);
            L.Tf.assign(eo.Tf.begin() + n0, eo.Tf.begin() + n0 + Ni);
            L.decision.assign(eo.decision.begin() + n0, eo.decision.begin() + n0 + Ni);
            it.R->levels.push_back(std::move(L));
        }
        // a9: column norms of X = V_m Y for every (pencil, shift) group of the level
        if (do_proj && N > 0) {
            std::vector<ProjGroup> gt;
            std::vector<int64_t> srccol;
            std::vector<std::pair<int, std::vector<int64_t>>> gsq;   // (pencil, rows) per group
            int64_t scr_need = 0;
            for (int i = 0; i < nb; ++i) {
                auto& it = items[i];
                if (k > it.R->K) continue;
                std::vector<std::vector<int64_t>> by((size_t)it.R->shifts.size());
                for (int64_t r = first[i]; r < first[i + 1]; ++r) by[used[r]].push_back(r);
                for (size_t s = 0; s < by.size(); ++s) {
                    if (by[s].empty()) continue;
                    ProjGroup pg{};
                    pg.n = it.p->n;
                    pg.m = it.R->shifts[s]->m_eff;
                    pg.V = it.R->shifts[s]->V;
                    pg.ldv = it.p->n;
                    pg.ldy = m;
                    pg.c = 2 * (int64_t)by[s].size();
                    project_group_shape(pg);
                    gt.push_back(pg);
                    for (int64_t r : by[s]) {
                        srccol.push_back(2 * r);
                        srccol.push_back(2 * r + 1);
                    }
                    scr_need += project_scratch_elems(pg.n, pg.c);
                    gsq.emplace_back(i, by[s]);
                }
            }
            const int64_t ncol = (int64_t)srccol.size(), ng = (int64_t)gt.size();
            if (mixed_proj) {
                // reduced-precision projections: one launch per group (outside the graph)
                std::vector<double> nh;
                SIMM_TRY(pe.Y.alloc(sizeof(cplx) * (size_t)ncol * m, st));
                SIMM_TRY(pe.src.alloc(sizeof(int64_t) * (size_t)ncol, st));
                SIMM_HIP_TRY(hipMemcpyAsync(pe.src.p, srccol.data(), sizeof(int64_t) * ncol, hipMemcpyHostToDevice, st));
                GatherDesc hd{main_eval.sums, m, pe.src.as<int64_t>(), nullptr, pe.Y.as<cplx>()};
                DevBuf db;
                SIMM_TRY(db.alloc(sizeof(GatherDesc) + sizeof(int64_t), st));
                int64_t* ncd = reinterpret_cast<int64_t*>(db.as<char>() + sizeof(GatherDesc));
                hd.ncols = ncd;
                SIMM_HIP_TRY(hipMemcpyAsync(db.p, &hd, sizeof(GatherDesc), hipMemcpyHostToDevice, st));
                SIMM_HIP_TRY(hipMemcpyAsync(ncd, &ncol, sizeof(int64_t), hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_gather_cols, dim3(1024), dim3(128), 0, st, db.as<const GatherDesc>());
                SIMM_HIP_TRY(hipGetLastError());
                SIMM_TRY(pe.norms.alloc(sizeof(double) * (size_t)ncol, st));
                int64_t col0 = 0;
                const int prec = (k <= 2) ? SIMM_PROJ_BF16 : SIMM_PROJ_FP32;
                for (auto& pg : gt) {
                    const int64_t se = project_scratch_elems(pg.n, pg.c);
                    SIMM_TRY(pe.scr.alloc(sizeof(double) * (size_t)se, st));
                    SIMM_TRY(project(pg.n, pg.m, pg.V, pg.ldv, pe.Y.as<cplx>() + col0 * m, m, pg.c, nullptr,
                                     pe.norms.as<double>() + col0, pe.scr.as<double>(), se, prec, st));
                    col0 += pg.c;
                }
                nh.assign((size_t)ncol, 0.0);
                SIMM_HIP_TRY(hipMemcpyAsync(nh.data(), pe.norms.p, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
                SIMM_HIP_TRY(hipStreamSynchronize(st));
                int64_t c0 = 0;
                for (auto& gs : gsq) {
                    LevelRec& L = items[gs.first].R->levels.back();
                    for (size_t q = 0; q < gs.second.size(); ++q)
                        L.full_indicator[gs.second[q] - first[gs.first]] = nh[c0 + 2 * q + 1] / nh[c0 + 2 * q];
                    c0 += 2 * (int64_t)gs.second.size();
                }
            } else {
                // buffers (pointers live in the device tables, so growth needs no new graph)
                if (ng > pe.gcap) {
                    (void)hipFree(pe.tab);
                    pe.tab = nullptr;
                    pe.graph.reset();
                    pe.gcap = std::max<int64_t>(64, ng * 2);
                    SIMM_HIP_TRY(hipMalloc(&pe.tab, 512 + sizeof(ProjGroup) * (size_t)pe.gcap));
                    pe.desc = reinterpret_cast<GatherDesc*>(pe.tab);
                    pe.counts = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(pe.tab) + 256);
                    pe.groups = reinterpret_cast<ProjGroup*>(reinterpret_cast<char*>(pe.tab) + 512);
                }
                SIMM_TRY(pe.Y.alloc(sizeof(cplx) * (size_t)ncol * m, st));
                SIMM_TRY(pe.src.alloc(sizeof(int64_t) * (size_t)ncol, st));
                SIMM_TRY(pe.scr.alloc(sizeof(double) * (size_t)scr_need, st));
                SIMM_TRY(pe.norms.alloc(sizeof(double) * (size_t)ncol, st));
                int64_t col0 = 0, sc0 = 0;
                int64_t tiles = 0;
                for (auto& pg : gt) {
                    pg.Y = pe.Y.as<cplx>() + col0 * m;
                    pg.colpart = pe.scr.as<double>() + sc0;
                    pg.part = pg.colpart + 2 * pg.gx * pg.c;
                    pg.norms = pe.norms.as<double>() + col0;
                    col0 += pg.c;
                    sc0 += project_scratch_elems(pg.n, pg.c);
                    tiles += pg.gx * pg.gy;
                }
                GatherDesc hd{main_eval.sums, m, pe.src.as<int64_t>(), pe.counts, pe.Y.as<cplx>()};
                const int64_t cnt[2] = {ncol, ng};
                SIMM_HIP_TRY(hipMemcpyAsync(pe.src.p, srccol.data(), sizeof(int64_t) * ncol, hipMemcpyHostToDevice, st));
                SIMM_HIP_TRY(hipMemcpyAsync(pe.desc, &hd, sizeof(GatherDesc), hipMemcpyHostToDevice, st));
                SIMM_HIP_TRY(hipMemcpyAsync(pe.counts, cnt, sizeof(cnt), hipMemcpyHostToDevice, st));
                SIMM_HIP_TRY(hipMemcpyAsync(pe.groups, gt.data(), sizeof(ProjGroup) * ng, hipMemcpyHostToDevice, st));
                const auto key = std::make_tuple(mmax, log2_bucket(tiles));
                int G = 0;
                {
                    std::lock_guard<std::mutex> lk(g_tune.mu);
                    auto itc = g_tune.proj.find(key);
                    if (itc != g_tune.proj.end()) G = itc->second;
                }
                if (G == 0) {
                    float best = 1e30f;
                    for (int cand : {256, 512, 1024, 2048}) {
                        if (cand > 8 * tiles && cand > 256) break;
                        SIMM_TRY(pe.capture(cand, st));
                        hipEvent_t a, b;
                        SIMM_HIP_TRY(hipEventCreate(&a));
                        SIMM_HIP_TRY(hipEventCreate(&b));
                        SIMM_HIP_TRY(hipEventRecord(a, st));
                        SIMM_TRY(pe.graph.launch(st));
                        SIMM_HIP_TRY(hipEventRecord(b, st));
                        SIMM_HIP_TRY(hipEventSynchronize(b));
                        float ms = 0;
                        (void)hipEventElapsedTime(&ms, a, b);
                        (void)hipEventDestroy(a);
                        (void)hipEventDestroy(b);
                        if (ms < best) {
                            best = ms;
                            G = cand;
                        }
                    }
                    std::lock_guard<std::mutex> lk(g_tune.mu);
                    g_tune.proj[key] = G;
                    g_tune.trials += 1;
                }
                if (pe.grid != G || !pe.graph.exec) SIMM_TRY(pe.capture(G, st));
                SIMM_TRY(pe.graph.launch(st));
                std::vector<double> nh((size_t)ncol);
                SIMM_HIP_TRY(hipMemcpyAsync(nh.data(), pe.norms.p, sizeof(double) * ncol, hipMemcpyDeviceToHost, st));
                SIMM_HIP_TRY(hipStreamSynchronize(st));
                int64_t c0 = 0;
                for (auto& gs : gsq) {
                    LevelRec& L = items[gs.first].R->levels.back();
                    for (size_t q = 0; q < gs.second.size(); ++q)
                        L.full_indicator[gs.second[q] - first[gs.first]] = nh[c0 + 2 * q + 1] / nh[c0 + 2 * q];
                    c0 += 2 * (int64_t)gs.second.size();
                }
            }
        }
        // children of the marked squares (each pencil's squares in (iy, ix) order)
        for (int i = 0; i < nb; ++i) {
            auto& it = items[i];
            if (k >= it.R->K) continue;
            std::vector<Sq> nxt;
            for (int64_t r = first[i]; r < first[i + 1]; ++r) {
                if (eo.decision[r] == SIMM_REJECTED) continue;
                const Sq& q = it.cur[r - first[i]];
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) nxt.push_back({2 * q.ix + a, 2 * q.iy + b, used[r]});
            }
            std::stable_sort(nxt.begin(), nxt.end(), [](const Sq& u, const Sq& v) {
                if (u.iy != v.iy) return u.iy < v.iy;
                return u.ix < v.ix;
            });
            it.cur.swap(nxt);
        }
    }
    return SIMM_OK;
}

simm_status to_device_vec(const double* src, int32_t mem, int64_t count, DevBuf& buf, const cplx** out,
                          hipStream_t st) {
    if (mem == SIMM_MEM_DEVICE) {
        *out = reinterpret_cast<const cplx*>(src);
        return SIMM_OK;
    }
    if (mem != SIMM_MEM_HOST) {
        set_error("mem must be SIMM_MEM_HOST or SIMM_MEM_DEVICE");
        return SIMM_EINVAL;
    }
    if (!finite_c(src, 2 * count)) {
        set_error("input vector has NaN/Inf");
        return SIMM_EINVAL;
    }
    SIMM_TRY(buf.alloc(sizeof(cplx) * (size_t)count, st));
    SIMM_HIP_TRY(hipMemcpyAsync(buf.p, src, sizeof(cplx) * (size_t)count, hipMemcpyHostToDevice, st));
    *out = buf.as<const cplx>();
    return SIMM_OK;
}

// Multiplicities (Sec. 3.4) of the clusters of a finished run: see simm_multiplicities.
constexpr int MULT_WORKERS = 4;

simm_status multiplicities(simm_result_s* R, const cplx* F, int k, double rel_tol, hipStream_t st, int32_t* mult,
                           double* sv) {
    const int64_t ncl = (int64_t)R->clusters.size();
    if (ncl == 0) return SIMM_OK;
    simm_pencil_s* p = R->pencil;
    const simm_params* prm = &R->prm;
    const int64_t n = p->n;
    const int m = prm->m;
    const LevelRec& last = R->levels.back();
    Rule rule;
    SIMM_TRY(rule.make(prm->gauss_per_edge, st));
    // X: n x (ncl k), column c k + i = P f_i of cluster c
    DevBuf xb, gb;
    SIMM_TRY(xb.alloc(sizeof(cplx) * (size_t)n * ncl * k, st));
    SIMM_HIP_TRY(hipMemsetAsync(xb.p, 0, sizeof(cplx) * (size_t)n * ncl * k, st));
    std::vector<int> used;
    for (const auto& c : R->clusters)
        for (int64_t q : c.members) used.push_back(last.shift[q]);
    std::sort(used.begin(), used.end());
    used.erase(std::unique(used.begin(), used.end()), used.end());
    // per shift: the squares of every cluster tested with it, grouped by cluster
    struct ShiftSquares {
        std::vector<int64_t> regs, off{0}, idx;
        DevBuf ib;
    };
    std::vector<ShiftSquares> sq(used.size());
    bool any_mixed = false;
    for (size_t u = 0; u < used.size(); ++u) {
        auto& q = sq[u];
        for (const auto& c : R->clusters) {
            for (int64_t m_ : c.members)
                if (last.shift[m_] == used[u]) {
                    q.idx.push_back((int64_t)q.regs.size() / 4);
                    q.regs.insert(q.regs.end(), {(int64_t)R->K, last.ix[m_], last.iy[m_], 0});
                }
            q.off.push_back((int64_t)q.idx.size());
        }
        SIMM_TRY(q.ib.alloc(sizeof(int64_t) * (q.off.size() + q.idx.size()), st));
        SIMM_HIP_TRY(hipMemcpyAsync(q.ib.p, q.off.data(), sizeof(int64_t) * q.off.size(), hipMemcpyHostToDevice, st));
        SIMM_HIP_TRY(hipMemcpyAsync(q.ib.as<int64_t>() + q.off.size(), q.idx.data(), sizeof(int64_t) * q.idx.size(),
                                    hipMemcpyHostToDevice, st));
        any_mixed = any_mixed || R->shifts[used[u]]->mixed;
    }
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    // The k Krylov spaces of a shift are independent.  They go in blocks of NB consecutive
    // start vectors whose spaces advance in lockstep (one multi-column application of M
    // per step), block b to worker b % W (a host thread with a stream of its own, the
    // factor's per-application buffers and shift objects whose basis and Schur buffers it
    // reuses), shifts in order, so column i of X receives its terms in the one-worker
    // order.  Refined (mixed-precision) shifts share one refinement state per shift: one
    // worker and one space at a time then.
    int NB = 1;
    if (!any_mixed) {
        NB = 4;
        for (int u : used) NB = std::min(NB, spike_max_nrhs(R->shifts[u]->spike));
        NB = std::max(1, std::min(NB, k));
    }
    const int nblocks = (k + NB - 1) / NB;
    const int W = any_mixed ? 1 : std::min(nblocks, MULT_WORKERS);
    struct Worker {
        hipStream_t st = nullptr;
        simm_shift_s kv[4];
        DevBuf tb, yb, sb;
        simm_status rc = SIMM_OK;
        std::string msg;
    };
    std::vector<Worker> wk((size_t)W);
    struct StreamRelease {
        std::vector<Worker>* w;
        ~StreamRelease() {
            for (auto& x : *w)
                if (x.st) {
                    (void)hipStreamSynchronize(x.st);
                    release_stream_buffers(x.st);
                    (void)hipStreamSynchronize(x.st);
                    (void)hipStreamDestroy(x.st);
                }
        }
    } stream_release{&wk};
    int64_t nsq_max = 1;
    for (auto& q : sq) nsq_max = std::max<int64_t>(nsq_max, (int64_t)q.idx.size());
    for (auto& x : wk) {
        SIMM_HIP_TRY(hipStreamCreateWithFlags(&x.st, hipStreamNonBlocking));
        SIMM_TRY(x.tb.alloc(sizeof(cplx) * (size_t)n * ncl, x.st));
        SIMM_TRY(x.yb.alloc(sizeof(cplx) * (size_t)m * ncl, x.st));
        SIMM_TRY(x.sb.alloc(sizeof(cplx) * (size_t)nsq_max * 2 * m, x.st));
    }
    SIMM_HIP_TRY(hipStreamSynchronize(st));   // X zeroed on st before the workers add to it
    int dev = 0;
    SIMM_HIP_TRY(hipGetDevice(&dev));
    auto work = [&](int w) {
        Worker& x = wk[(size_t)w];
        (void)hipSetDevice(dev);
        auto body = [&]() -> simm_status {
            for (size_t u = 0; u < used.size(); ++u) {
                const simm_shift_s* base = R->shifts[used[u]].get();
                auto& q = sq[u];
                const int64_t* offd = q.ib.as<int64_t>();
                const int64_t* idxd = offd + q.off.size();
                SpikeFactor clone{};
                const bool own = W > 1 || NB > 1;
                if (own) SIMM_TRY(spike_clone_scratch(base->spike, clone, x.st, true, NB));
                for (int b = w; b < nblocks; b += W) {
                    // Krylov spaces of f_i, i in block b, on the shift's factor
                    const int i0 = b * NB, nb = std::min(NB, k - i0);
                    simm_shift_s* kvp[4];
                    for (int r = 0; r < nb; ++r) {
                        x.kv[r].borrow_factor_of(base);
                        if (own) x.kv[r].spike = clone;
                        kvp[r] = &x.kv[r];
                    }
                    if (nb == 1) SIMM_TRY(krylov_shift(kvp[0], F + (int64_t)i0 * n, m, x.st, nullptr));
                    else SIMM_TRY(krylov_block(kvp, nb, F + (int64_t)i0 * n, n, m, x.st));
                    for (int r = 0; r < nb; ++r) {
                        simm_shift_s& kv = x.kv[r];
                        const int i = i0 + r;
                        EvalOut eo;
                        SIMM_TRY(evaluate({&kv}, q.regs, prm, rule, x.st, eo, x.sb.as<cplx>(), m));
                        SIMM_TRY(cluster_sums(x.sb.as<cplx>(), m, offd, idxd, ncl, kv.m_eff, x.yb.as<cplx>(), m, x.st));
                        SIMM_TRY(project(n, kv.m_eff, kv.V, n, x.yb.as<cplx>(), m, ncl, x.tb.as<cplx>(), nullptr,
                                         nullptr, 0, SIMM_PROJ_FP64, x.st));
                        SIMM_TRY(accum_cols(n, ncl, x.tb.as<cplx>(), xb.as<cplx>() + (int64_t)i * n, (int64_t)k * n,
                                            x.st));
                    }
                }
                if (own) {
                    int e = 0;
                    SIMM_HIP_TRY(hipMemcpyAsync(&e, clone.err, sizeof(int), hipMemcpyDeviceToHost, x.st));
                    SIMM_HIP_TRY(hipStreamSynchronize(x.st));
                    spike_release_ordered(clone, x.st);
                    if (e) {
                        set_error("partitioned sweep: a chunk-chain barrier timed out");
                        return SIMM_EHIP;
                    }
                }
            }
            SIMM_HIP_TRY(hipStreamSynchronize(x.st));
            return SIMM_OK;
        };
        x.rc = body();
        if (x.rc != SIMM_OK) x.msg = simm_last_error();
    };
    {
        std::vector<std::thread> pool;
        for (int w = 1; w < W; ++w) pool.emplace_back(work, w);
        work(0);
        for (auto& t : pool) t.join();
    }
    for (auto& x : wk)
        if (x.rc != SIMM_OK) {
            set_error(x.msg);
            return x.rc;
        }
    SIMM_TRY(gb.alloc(sizeof(cplx) * (size_t)ncl * k * k, st));
    SIMM_TRY(gram(n, k, ncl, xb.as<cplx>(), gb.as<cplx>(), st));
    std::vector<cplx> G((size_t)ncl * k * k);
    SIMM_HIP_TRY(hipMemcpyAsync(G.data(), gb.p, sizeof(cplx) * G.size(), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    for (int64_t c = 0; c < ncl; ++c) {
        const std::vector<double> ev = hermitian_eigenvalues(k, G.data() + (size_t)c * k * k);
        int cnt = 0;
        const double s0 = std::sqrt(std::max(ev[0], 0.0));
        for (int i = 0; i < k; ++i) {
            const double si = std::sqrt(std::max(ev[i], 0.0));
            if (sv) sv[(size_t)c * k + i] = si;
            if (s0 > 0.0 && si > rel_tol * s0) ++cnt;
        }
        mult[c] = cnt;
    }
    return SIMM_OK;
}

// Adjoint gradient of J = sum_R ||x_R||^2 over the squares `regs` (see simm_gradient).
// The conjugate-transposed pencil (A^H, B^H) is factored once per shift at conj(sigma);
// each square gets one Krylov space of that pencil started from x_R, whose fine-rule
// solutions at the conjugated nodes approximate lambda_j = (A - z_j B)^{-H} x_R.  The
// squares of a shift are dealt round-robin to GRAD_WORKERS host threads, each with a
// stream, a copy of the factor's per-application buffers and its own accumulators
// (J, dJ/dp, the diagonal gradient); the accumulators are summed in worker order at
// the end, so the result does not depend on timing.
constexpr int GRAD_WORKERS = 4;

simm_status gradient(const std::vector<simm_shift_s*>& shifts, const std::vector<int64_t>& regs,
                     const simm_params* prm, int kl1, int ku1, const cplx* A1, double* J, double* dJdp, cplx* grad,
                     hipStream_t st) {
    simm_pencil_s* p = shifts[0]->p;
    const int64_t n = p->n;
    const int64_t N = (int64_t)regs.size() / 4;
    const int g = prm->gauss_per_edge;
    const int nf = 8 * g;
    constexpr int LDY = 128;
    const bool adjoint = (A1 != nullptr || grad != nullptr);
    Rule rule;
    SIMM_TRY(rule.make(g, st));
    int mmax = 1;
    for (auto* s : shifts) mmax = std::max(mmax, s->m_eff);
    DevBuf sumsb;
    SIMM_TRY(sumsb.alloc(sizeof(cplx) * (size_t)N * 2 * mmax, st));
    cplx* sums = sumsb.as<cplx>();
    EvalOut eo;
    SIMM_TRY(evaluate(shifts, regs, prm, rule, st, eo, sums, mmax));
    // the squares' own solves must be resolved (Definition 3.1): an unresolved square's
    // sums, and so its x_R, are not accurate
    for (int64_t r = 0; r < N; ++r)
        if (eo.decision[r] == SIMM_UNRESOLVED) {
            char msg[200];
            std::snprintf(msg, sizeof msg, "square %lld is not resolved by its shift: residual %.3g > eps0 = %.3g "
                          "(raise m)", (long long)r, eo.rho[r], prm->eps0);
            set_error(msg);
            return SIMM_EUNRESOLVED;
        }
    IndicatorParams ip;
    ip.x0 = prm->x0;
    ip.y0 = prm->y0;
    ip.w1 = (prm->x1 - prm->x0) / prm->n1;
    ip.eps0 = prm->eps0;
    ip.delta0 = prm->delta0;
    ip.tau = prm->tau;

    // the conjugate-transposed pencil
    simm_pencil_s adj;
    struct AdjRelease {
        simm_pencil_s* q;
        ~AdjRelease() {
            (void)hipFree(q->A);
            (void)hipFree(q->B);
        }
    } adj_release{&adj};
    adj.n = n;
    adj.kla = p->kua;
    adj.kua = p->kla;
    adj.klb = p->B ? p->kub : 0;
    adj.kub = p->B ? p->klb : 0;
    adj.dev = p->dev;
    if (adjoint) {
        SIMM_TRY(dalloc(&adj.A, (size_t)(p->kla + p->kua + 1) * n));
        SIMM_TRY(conj_transpose_band(n, p->kla, p->kua, p->A, adj.A, st));
        if (p->B) {
            SIMM_TRY(dalloc(&adj.B, (size_t)(p->klb + p->kub + 1) * n));
            SIMM_TRY(conj_transpose_band(n, p->klb, p->kub, p->B, adj.B, st));
        }
    }

    // per-worker buffers (allocated on st, used on the worker streams after st is
    // synchronized, freed on st after the workers' streams are)
    struct Worker {
        hipStream_t st = nullptr;
        SpikeFactor sp;
        bool has_sp = false;
        simm_shift_s kv[4];   // the adjoint spaces of a block of squares (bases and Schur buffers kept)
        DevBuf xb, zb, z1b, yb, cwb, kb, pb, rhob;
        simm_status rc = SIMM_OK;
        std::string msg;
    };
    const int W = adjoint ? GRAD_WORKERS : 1;
    DevBuf accb, wb, gradsb;   // declared before the workers: freed after their streams drain
    std::vector<Worker> wk((size_t)W);
    struct StreamRelease {
        std::vector<Worker>* w;
        ~StreamRelease() {
            for (auto& x : *w) {
                if (x.st) (void)hipStreamSynchronize(x.st);
                if (x.has_sp) spike_release(x.sp);
            }
            for (auto& x : *w)
                if (x.st) {
                    release_stream_buffers(x.st);
                    (void)hipStreamSynchronize(x.st);
                    (void)hipStreamDestroy(x.st);
                }
        }
    } stream_release{&wk};
    SIMM_TRY(accb.alloc(sizeof(double) * 2 * W, st));
    SIMM_HIP_TRY(hipMemsetAsync(accb.p, 0, sizeof(double) * 2 * W, st));
    if (A1) SIMM_TRY(wb.alloc(sizeof(cplx) * (size_t)n * mmax, st));
    if (grad) {
        SIMM_TRY(gradsb.alloc(sizeof(cplx) * (size_t)n * W, st));
        SIMM_HIP_TRY(hipMemsetAsync(gradsb.p, 0, sizeof(cplx) * (size_t)n * W, st));
    }
    for (int w = 0; w < W; ++w) {
        Worker& x = wk[(size_t)w];
        SIMM_HIP_TRY(hipStreamCreateWithFlags(&x.st, hipStreamNonBlocking));
        SIMM_TRY(x.xb.alloc(sizeof(cplx) * (size_t)n * 4, st));   // x_R of up to four squares
        if (A1) SIMM_TRY(x.z1b.alloc(sizeof(cplx) * (size_t)n * 128, st));
        if (grad) SIMM_TRY(x.zb.alloc(sizeof(cplx) * (size_t)n * 128, st));
        SIMM_TRY(x.yb.alloc(sizeof(cplx) * (size_t)2 * nf * LDY, st));
        SIMM_TRY(x.cwb.alloc(sizeof(cplx) * (size_t)nf, st));
        SIMM_TRY(x.rhob.alloc(sizeof(double) * (size_t)nf, st));
        SIMM_TRY(x.kb.alloc(sizeof(cplx) * (size_t)128 * 128, st));
        SIMM_TRY(x.pb.alloc(sizeof(cplx) * (size_t)grad_part_elems(n), st));
    }
    int dev = 0;
    SIMM_HIP_TRY(hipGetDevice(&dev));

    std::vector<int> used;
    for (int64_t r = 0; r < N; ++r) used.push_back((int)regs[4 * r + 3]);
    std::sort(used.begin(), used.end());
    used.erase(std::unique(used.begin(), used.end()), used.end());
    int64_t next_worker = 0;   // squares are dealt to workers in order across shifts
    for (int si : used) {
        simm_shift_s* fs = shifts[si];
        const int mf = fs->m_eff;
        std::vector<int64_t> rs;   // this shift's squares whose s_f does not vanish
        for (int64_t r = 0; r < N; ++r)
            if (regs[4 * r + 3] == si && eo.nsf[r] > 0.0) rs.push_back(r);
        if (rs.empty()) continue;
        if (!adjoint) {
            // J alone: ||x_R||^2 of every square
            Worker& x = wk[0];
            for (int64_t r : rs) {
                SIMM_TRY(project(n, mf, fs->V, n, sums + (2 * r + 1) * mmax, mmax, 1, x.xb.as<cplx>(), nullptr,
                                 nullptr, 0, SIMM_PROJ_FP64, st));
                SIMM_TRY(grad_rowdot(n, 0, nullptr, n, nullptr, nullptr, n, x.xb.as<cplx>(), nullptr,
                                     x.pb.as<cplx>(), accb.as<double>(), st));
            }
            continue;
        }
        std::unique_ptr<simm_shift_s> af;
        SIMM_TRY(factor_shift(&adj, conj(fs->sigma), st, af));
        SIMM_TRY(prepare_sweeps(af.get(), st));
        if (A1)
            for (int k = 0; k < mf; ++k)
                SIMM_TRY(prepare_input(n, fs->V + (int64_t)k * n, A1, kl1, ku1, nullptr, nullptr,
                                       wb.as<cplx>() + (int64_t)k * n, nullptr, st));
        // squares in blocks of NB whose adjoint spaces advance in lockstep (one pass over
        // the adjoint factor per step for all of them)
        const int NB = af->mixed ? 1 : std::min(4, spike_max_nrhs(af->spike));
        for (auto& x : wk) {
            if (x.has_sp) spike_release(x.sp);
            x.has_sp = false;
            SIMM_TRY(spike_clone_scratch(af->spike, x.sp, st, false, NB));
            x.has_sp = true;
        }
        SIMM_HIP_TRY(hipStreamSynchronize(st));
        const ShiftDev fd = shift_dev(fs);
        // a block of squares on worker x: their x_R and adjoint Krylov spaces (in lockstep),
        // then per square K_R, Z, Z1 and the row dots
        auto square_rest = [&](Worker& x, int w, int64_t r, simm_shift_s& kv, const cplx* xr) -> simm_status {
            const int ma = kv.m_eff;
            if (ma > 128) {
                set_error("Krylov dimension above 128");
                return SIMM_EUNSUPPORTED;
            }
            const ShiftDev ad = shift_dev(&kv);
            const int level = (int)regs[4 * r];
            cplx* Yf = x.yb.as<cplx>();
            cplx* Ya = Yf + (size_t)nf * LDY;
            SIMM_TRY(fine_solutions(fd, ip, rule.dev, level, regs[4 * r + 1], regs[4 * r + 2], false, Yf, LDY,
                                    x.cwb.as<cplx>(), nullptr, x.st));
            SIMM_TRY(fine_solutions(ad, ip, rule.dev, level, regs[4 * r + 1], regs[4 * r + 2], true, Ya, LDY,
                                    nullptr, x.rhob.as<double>(), x.st));
            SIMM_TRY(grad_kmat(nf, Yf, Ya, LDY, x.cwb.as<cplx>(), mf, ma, x.kb.as<cplx>(), x.st));
            if (grad)
                SIMM_TRY(project(n, mf, fs->V, n, x.kb.as<cplx>(), mf, ma, x.zb.as<cplx>(), nullptr, nullptr, 0,
                                 SIMM_PROJ_FP64, x.st));
            if (A1)
                SIMM_TRY(project(n, mf, wb.as<cplx>(), n, x.kb.as<cplx>(), mf, ma, x.z1b.as<cplx>(), nullptr,
                                 nullptr, 0, SIMM_PROJ_FP64, x.st));
            SIMM_TRY(grad_rowdot(n, ma, kv.V, n, grad ? x.zb.as<cplx>() : nullptr, A1 ? x.z1b.as<cplx>() : nullptr,
                                 n, xr, grad ? gradsb.as<cplx>() + (int64_t)w * n : nullptr,
                                 x.pb.as<cplx>(), accb.as<double>() + 2 * w, x.st));
            std::vector<double> rho_adj((size_t)nf);
            SIMM_HIP_TRY(hipMemcpyAsync(rho_adj.data(), x.rhob.p, sizeof(double) * nf, hipMemcpyDeviceToHost, x.st));
            SIMM_HIP_TRY(hipStreamSynchronize(x.st));   // kv's buffers are freed at scope exit
            // the adjoint solutions must be resolved in their Krylov space like the forward
            // ones (Definition 3.1 with eq. (error) at the conjugated nodes)
            const double rmax = *std::max_element(rho_adj.begin(), rho_adj.end());
            if (!(rmax <= prm->eps0)) {
                char msg[200];
                std::snprintf(msg, sizeof msg,
                              "adjoint Krylov space of square %lld not resolved: residual %.3g > eps0 = %.3g "
                              "(raise m)", (long long)r, rmax, prm->eps0);
                set_error(msg);
                return SIMM_EUNRESOLVED;
            }
            return SIMM_OK;
        };
        auto block = [&](Worker& x, int w, const int64_t* sq, int nb) -> simm_status {
            simm_shift_s* kvp[4];
            for (int b = 0; b < nb; ++b) {
                SIMM_TRY(project(n, mf, fs->V, n, sums + (2 * sq[b] + 1) * mmax, mmax, 1, x.xb.as<cplx>() + b * n,
                                 nullptr, nullptr, 0, SIMM_PROJ_FP64, x.st));
                simm_shift_s& kv = x.kv[b];
                kv.p = &adj;
                kv.sigma = af->sigma;
                kv.kl = af->kl;
                kv.ku = af->ku;
                kv.AB = af->AB;
                kv.ipiv = af->ipiv;
                kv.LP = af->LP;
                kv.spike = x.sp;
                kv.sweeps_ready = true;
                kv.factor_borrowed = true;
                kvp[b] = &kv;
            }
            if (nb == 1) SIMM_TRY(krylov_shift(kvp[0], x.xb.as<cplx>(), fs->m, x.st, nullptr));
            else SIMM_TRY(krylov_block(kvp, nb, x.xb.as<cplx>(), n, fs->m, x.st));
            for (int b = 0; b < nb; ++b) SIMM_TRY(square_rest(x, w, sq[b], x.kv[b], x.xb.as<cplx>() + b * n));
            return SIMM_OK;
        };
        // blocks of NB consecutive squares, dealt to the workers in turn across shifts
        const int64_t nblocks = ((int64_t)rs.size() + NB - 1) / NB;
        const int64_t first = next_worker;
        auto run_worker = [&](int w) {
            (void)hipSetDevice(dev);
            Worker& x = wk[(size_t)w];
            for (int64_t q = 0; q < nblocks; ++q) {
                if ((int)((first + q) % W) != w) continue;
                const int64_t k0 = q * NB;
                const int nb = (int)std::min<int64_t>(NB, (int64_t)rs.size() - k0);
                const simm_status rc = block(x, w, rs.data() + k0, nb);
                if (rc != SIMM_OK) {
                    x.rc = rc;
                    x.msg = simm_last_error();
                    return;
                }
            }
        };
        std::vector<std::thread> pool;
        for (int w = 1; w < W; ++w) pool.emplace_back(run_worker, w);
        run_worker(0);
        for (auto& t : pool) t.join();
        next_worker = (first + nblocks) % W;
        for (auto& x : wk) {
            if (x.rc != SIMM_OK) {
                for (auto& y : wk) (void)hipStreamSynchronize(y.st);   // before af and the buffers go
                set_error(x.msg);
                return x.rc;
            }
        }
    }
    SIMM_TRY(grad_combine(n, W, gradsb.as<cplx>(), grad, accb.as<double>(), st));
    double acc[2] = {0.0, 0.0};
    SIMM_HIP_TRY(hipMemcpyAsync(acc, accb.p, sizeof(acc), hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    *J = acc[0];
    if (dJdp) *dJdp = acc[1];
    return SIMM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// exported C ABI
// ---------------------------------------------------------------------------
// Scratch of simm_project_noalloc: the per-64-row partial column norms and their
// group sums, for callers that cannot allocate device memory.  Each device holds its
// own copy of this array for the life of the process; its device address is looked
// up once per device (in host code the array's name is not a device address) and
// kept.  Calls that overlap on one device share it.
namespace {
constexpr int64_t kNoAllocScratchDoubles = (int64_t)2 << 20;   // 16 MiB
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;

simm_status noalloc_scratch(double** out) {
    int dev = 0;
    SIMM_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        double* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return SIMM_EHIP;
        }
        it = g_scratch_addr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return SIMM_OK;
}
}  // namespace

extern "C" {

const char* simm_last_error(void) { return g_err.c_str(); }
int32_t simm_version(void) { return 1; }

simm_status simm_params_default(simm_params* p) {
    if (!p) return SIMM_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->x0 = -1;
    p->x1 = 1;
    p->y0 = -1;
    p->y1 = 1;
    p->n1 = 8;
    p->gauss_per_edge = 8;
    p->m = 50;
    p->levels = 0;
    p->h0 = 1e-6;
    p->eps0 = 1e-8;
    p->delta0 = 0.05;
    p->tau = 1e-8;
    p->max_regions_per_level = (int64_t)1 << 22;
    p->flags = 0;
    p->lookahead = 0;
    p->precision = SIMM_PREC_FP64;
    return SIMM_OK;
}

simm_status simm_pencil_create_banded(int64_t n, int32_t kl_a, int32_t ku_a, const double* a_band, int32_t kl_b,
                                      int32_t ku_b, const double* b_band, int32_t mem, void* hip_stream,
                                      simm_pencil* out) {
    clear_error();
    if (!out) return SIMM_EINVAL;
    *out = nullptr;
    if (n < 1 || kl_a < 0 || ku_a < 0 || !a_band || (b_band && (kl_b < 0 || ku_b < 0))) {
        set_error("bad pencil arguments");
        return SIMM_EINVAL;
    }
    if (mem != SIMM_MEM_HOST && mem != SIMM_MEM_DEVICE) {
        set_error("mem must be SIMM_MEM_HOST or SIMM_MEM_DEVICE");
        return SIMM_EINVAL;
    }
    SIMM_TRY(check_device());
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t na = (size_t)(kl_a + ku_a + 1) * n;
    const size_t nbb = b_band ? (size_t)(kl_b + ku_b + 1) * n : 0;
    if (mem == SIMM_MEM_HOST) {
        if (!finite_c(a_band, 2 * (int64_t)na) || (b_band && !finite_c(b_band, 2 * (int64_t)nbb))) {
            set_error("pencil has NaN/Inf entries");
            return SIMM_EINVAL;
        }
    }
    auto p = std::make_unique<simm_pencil_s>();
    p->n = n;
    p->kla = kl_a;
    p->kua = ku_a;
    p->klb = b_band ? kl_b : 0;
    p->kub = b_band ? ku_b : 0;
    SIMM_TRY(dalloc(&p->A, na));
    const hipMemcpyKind kind = (mem == SIMM_MEM_HOST) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    SIMM_HIP_TRY(hipMemcpyAsync(p->A, a_band, sizeof(cplx) * na, kind, st));
    if (b_band) {
        SIMM_TRY(dalloc(&p->B, nbb));
        SIMM_HIP_TRY(hipMemcpyAsync(p->B, b_band, sizeof(cplx) * nbb, kind, st));
    }
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    // A band that the shift factors partition uses the pooled spike streams: made now,
    // before any stream of a run, they spread evenly over the hardware queues (the HIP
    // runtime gives a new stream the queue that the fewest live streams use, so pooled
    // streams made while a run's streams live would leave the queues unevenly used, and
    // the worker streams made later would pile onto the least used one).
    if (part_block_len(n, std::max(p->kla, p->klb), std::max(p->kua, p->kub)) > 0) {
        hipStream_t pool[4] = {};
        SIMM_TRY(spike_streams(pool));
    }
    *out = p.release();
    return SIMM_OK;
}

simm_status simm_pencil_create_csr(int64_t n, const int64_t* a_rowptr, const int32_t* a_col, const double* a_val,
                                   const int64_t* b_rowptr, const int32_t* b_col, const double* b_val,
                                   void* hip_stream, simm_pencil* out) {
    clear_error();
    if (!out || n < 1 || !a_rowptr || !a_col || !a_val || (b_rowptr && (!b_col || !b_val))) {
        set_error("bad CSR arguments");
        return SIMM_EINVAL;
    }
    *out = nullptr;
    auto bw = [&](const int64_t* rp, const int32_t* ci, int* kl, int* ku) -> simm_status {
        *kl = 0;
        *ku = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (rp[i + 1] < rp[i]) return SIMM_EINVAL;
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
                const int64_t j = ci[q];
                if (j < 0 || j >= n) return SIMM_EINVAL;
                *kl = (int)std::max<int64_t>(*kl, i - j);
                *ku = (int)std::max<int64_t>(*ku, j - i);
            }
        }
        return SIMM_OK;
    };
    int kla, kua, klb = 0, kub = 0;
    if (bw(a_rowptr, a_col, &kla, &kua) != SIMM_OK || (b_rowptr && bw(b_rowptr, b_col, &klb, &kub) != SIMM_OK)) {
        set_error("malformed CSR structure");
        return SIMM_EINVAL;
    }
    if (std::max(kla, kua) > 4096 || std::max(klb, kub) > 4096) {
        set_error("half-bandwidth above 4096");
        return SIMM_EUNSUPPORTED;
    }
    auto to_band = [&](const int64_t* rp, const int32_t* ci, const double* v, int kl, int ku) {
        std::vector<double> band((size_t)2 * (kl + ku + 1) * n, 0.0);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
                const int64_t j = ci[q];
                const size_t at = 2 * ((size_t)(ku + i - j) + (size_t)j * (kl + ku + 1));
                band[at] += v[2 * q];
                band[at + 1] += v[2 * q + 1];
            }
        return band;
    };
    std::vector<double> ab = to_band(a_rowptr, a_col, a_val, kla, kua);
    std::vector<double> bb;
    if (b_rowptr) bb = to_band(b_rowptr, b_col, b_val, klb, kub);
    return simm_pencil_create_banded(n, kla, kua, ab.data(), klb, kub, b_rowptr ? bb.data() : nullptr,
                                     SIMM_MEM_HOST, hip_stream, out);
}

simm_status simm_pencil_info(simm_pencil p, int64_t* n, int32_t* kl, int32_t* ku) {
    if (!p) return SIMM_EINVAL;
    if (n) *n = p->n;
    if (kl) *kl = std::max(p->kla, p->klb);
    if (ku) *ku = std::max(p->kua, p->kub);
    return SIMM_OK;
}

void simm_pencil_destroy(simm_pencil p) {
    if (!p) return;
    (void)hipFree(p->A);
    (void)hipFree(p->B);
    delete p;
}

simm_status simm_shift_build(simm_pencil p, double sig_re, double sig_im, const double* f, int32_t f_mem, int32_t m,
                             int32_t precision, void* hip_stream, simm_shift* out) {
    clear_error();
    if (!out) return SIMM_EINVAL;
    *out = nullptr;
    if (!p || !f || !std::isfinite(sig_re) || !std::isfinite(sig_im)) {
        set_error("bad shift arguments");
        return SIMM_EINVAL;
    }
    if (m < 1 || m > p->n) {
        set_error("need 1 <= m <= n");
        return SIMM_EINVAL;
    }
    if (m > 128) {
        set_error("Krylov dimension above 128 is not supported");
        return SIMM_EUNSUPPORTED;
    }
    if (precision != SIMM_PREC_FP64 && precision != SIMM_PREC_MIXED) {
        set_error("precision must be SIMM_PREC_FP64 or SIMM_PREC_MIXED");
        return SIMM_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    DevBuf fb;
    const cplx* fd = nullptr;
    SIMM_TRY(to_device_vec(f, f_mem, p->n, fb, &fd, st));
    std::unique_ptr<simm_shift_s> s;
    SIMM_TRY(build_shift(p, cplx{sig_re, sig_im}, fd, m, st, s, nullptr, nullptr, precision));
    *out = s.release();
    return SIMM_OK;
}

simm_status simm_shift_from_hessenberg(double sig_re, double sig_im, double beta, const double* H, int32_t m_eff,
                                       void* hip_stream, simm_shift* out) {
    clear_error();
    if (!out) return SIMM_EINVAL;
    *out = nullptr;
    if (!H || !std::isfinite(sig_re) || !std::isfinite(sig_im) || !std::isfinite(beta) || !(beta > 0.0)) {
        set_error("bad shift arguments (H NULL, non-finite sigma, or beta not > 0)");
        return SIMM_EINVAL;
    }
    if (m_eff < 1) {
        set_error("need m_eff >= 1");
        return SIMM_EINVAL;
    }
    if (m_eff > 128) {
        set_error("Krylov dimension above 128 is not supported");
        return SIMM_EUNSUPPORTED;
    }
    const int64_t cnt = (int64_t)(m_eff + 1) * m_eff;
    if (!finite_c(H, 2 * cnt)) {
        set_error("H has NaN/Inf entries");
        return SIMM_EINVAL;
    }
    const cplx* Hc = reinterpret_cast<const cplx*>(H);
    for (int j = 0; j < m_eff; ++j)
        for (int i = j + 2; i <= m_eff; ++i)
            if (Hc[i + (int64_t)j * (m_eff + 1)].re != 0.0 || Hc[i + (int64_t)j * (m_eff + 1)].im != 0.0) {
                set_error("H is not upper Hessenberg");
                return SIMM_EINVAL;
            }
    SIMM_TRY(check_device());
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    auto s = std::make_unique<simm_shift_s>();
    s->sigma = cplx{sig_re, sig_im};
    s->m = s->m_eff = m_eff;
    s->beta = beta;
    s->factor_borrowed = true;   // no factor, sweep data or basis to free
    s->H_host.assign(Hc, Hc + cnt);
    s->h_last = cabs(s->H_host[m_eff + (size_t)(m_eff - 1) * (m_eff + 1)]);
    SIMM_TRY(dalloc(&s->H, (size_t)cnt));
    SIMM_HIP_TRY(hipMemcpyAsync(s->H, Hc, sizeof(cplx) * cnt, hipMemcpyHostToDevice, st));
    DevBuf status;
    SIMM_TRY(status.alloc(sizeof(int), st));
    SIMM_HIP_TRY(hipMemsetAsync(status.p, 0, sizeof(int), st));
    SIMM_TRY(schur_phase(s.get(), m_eff + 1, status.as<int>(), st));
    *out = s.release();
    return SIMM_OK;
}

simm_status simm_shift_info(simm_shift s, double* sigma, double* beta, int32_t* m_eff, double* H, double* ritz) {
    if (!s) return SIMM_EINVAL;
    if (sigma) {
        sigma[0] = s->sigma.re;
        sigma[1] = s->sigma.im;
    }
    if (beta) *beta = s->beta;
    if (m_eff) *m_eff = s->m_eff;
    if (H) std::memcpy(H, s->H_host.data(), sizeof(cplx) * s->H_host.size());
    if (ritz) std::memcpy(ritz, s->ritz.data(), sizeof(cplx) * s->ritz.size());
    return SIMM_OK;
}

simm_status simm_shift_basis(simm_shift s, double* V, int32_t mem, void* hip_stream) {
    clear_error();
    if (!s || !V) return SIMM_EINVAL;
    if (!s->has_factor()) {
        set_error("the shift's Krylov basis was released (SIMM_FLAG_RELEASE_FACTORS)");
        return SIMM_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const size_t cnt = (size_t)s->p->n * (s->m_eff + 1);
    SIMM_HIP_TRY(hipMemcpyAsync(V, s->V, sizeof(cplx) * cnt,
                                mem == SIMM_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    return SIMM_OK;
}

simm_status simm_shift_apply(simm_shift s, const double* x, double* y, int32_t mem, void* hip_stream) {
    clear_error();
    if (!s || !x || !y || x == y) {
        set_error("bad apply arguments");
        return SIMM_EINVAL;
    }
    if (!s->has_factor()) {
        set_error("the shift's factor was released (SIMM_FLAG_RELEASE_FACTORS)");
        return SIMM_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t n = s->p->n;
    DevBuf xb, ub, yb;
    const cplx* xd = nullptr;
    SIMM_TRY(to_device_vec(x, mem, n, xb, &xd, st));
    SIMM_TRY(ub.alloc(sizeof(cplx) * n, st));
    cplx* yd = reinterpret_cast<cplx*>(y);
    if (mem == SIMM_MEM_HOST) {
        SIMM_TRY(yb.alloc(sizeof(cplx) * n, st));
        yd = yb.as<cplx>();
    }
    SIMM_TRY(prepare_input(n, xd, s->p->B, s->p->klb, s->p->kub, nullptr, nullptr, ub.as<cplx>(), nullptr, st));
    ChainSlots slots;   // released (after a synchronize) when this returns
    SIMM_TRY(slots.acquire(spike_chain_weight(s->spike), st));
    SIMM_TRY(apply_inverse(s, ub.as<const cplx>(), yd, nullptr, st));
    if (mem == SIMM_MEM_HOST) SIMM_HIP_TRY(hipMemcpyAsync(y, yd, sizeof(cplx) * n, hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    return SIMM_OK;
}

simm_status simm_shift_apply_many(simm_shift s, const double* X, double* Y, int32_t k, int32_t mem,
                                  void* hip_stream) {
    clear_error();
    if (!s || !X || !Y || X == Y || k < 0) {
        set_error("bad apply arguments");
        return SIMM_EINVAL;
    }
    if (mem != SIMM_MEM_HOST && mem != SIMM_MEM_DEVICE) {
        set_error("mem must be SIMM_MEM_HOST or SIMM_MEM_DEVICE");
        return SIMM_EINVAL;
    }
    if (!s->has_factor()) {
        set_error("the shift's factor was released (SIMM_FLAG_RELEASE_FACTORS)");
        return SIMM_EINVAL;
    }
    if (k == 0) return SIMM_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t n = s->p->n, n16 = s->spike.n16;
    DevBuf xb, yb, ub;
    const cplx* xd = nullptr;
    SIMM_TRY(to_device_vec(X, mem, n * k, xb, &xd, st));
    cplx* yd = reinterpret_cast<cplx*>(Y);
    if (mem == SIMM_MEM_HOST) {
        SIMM_TRY(yb.alloc(sizeof(cplx) * (size_t)n * k, st));
        yd = yb.as<cplx>();
    }
    // up to four columns per pass over the factor (one at a time for a refined FP32 factor)
    const int nb = s->mixed ? 1 : std::min(4, spike_max_nrhs(s->spike));
    SpikeFactor clone{};
    struct CloneRelease {
        SpikeFactor* c;
        hipStream_t st;
        bool on = false;
        ~CloneRelease() {
            if (on) {
                (void)hipStreamSynchronize(st);
                spike_release_ordered(*c, st);
            }
        }
    } clone_release{&clone, st};
    if (nb > 1) {
        SIMM_TRY(spike_clone_scratch(s->spike, clone, st, true, nb));
        clone_release.on = true;
    }
    SIMM_TRY(ub.alloc(sizeof(cplx) * (size_t)n16 * nb, st));
    cplx* U = ub.as<cplx>();
    ChainSlots slots;   // released (after a synchronize) when this returns
    SIMM_TRY(slots.acquire(spike_chain_weight(s->spike), st));
    for (int c0 = 0; c0 < k;) {
        int nr = std::min(nb, k - c0);
        if (nr == 3) nr = 2;
        for (int r = 0; r < nr; ++r)
            SIMM_TRY(prepare_input(n, xd + (int64_t)(c0 + r) * n, s->p->B, s->p->klb, s->p->kub, nullptr, nullptr,
                                   U + r * n16, nullptr, st));
        if (nb == 1) SIMM_TRY(apply_inverse(s, U, yd + (int64_t)c0 * n, nullptr, st));
        else SIMM_TRY(spike_apply_nr(clone, U, n16, yd + (int64_t)c0 * n, n, nr, st));
        c0 += nr;
    }
    int err = 0;
    SIMM_HIP_TRY(hipMemcpyAsync(&err, nb > 1 ? clone.err : s->spike.err, sizeof(int), hipMemcpyDeviceToHost, st));
    if (mem == SIMM_MEM_HOST)
        SIMM_HIP_TRY(hipMemcpyAsync(Y, yd, sizeof(cplx) * (size_t)n * k, hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    if (err) {
        set_error("partitioned sweep: a chunk-chain barrier timed out");
        return SIMM_EHIP;
    }
    return SIMM_OK;
}

void simm_shift_destroy(simm_shift s) {
    if (s && !s->borrowed) delete s;
}

simm_status simm_cell_residuals(simm_shift s, int32_t level, const int64_t* squares, int64_t n_squares,
                                const simm_params* params, double* rho_max, int32_t mem, void* hip_stream) {
    clear_error();
    if (!s || !params || n_squares < 0 || (n_squares > 0 && (!squares || !rho_max)) || level < 1 || level > 60) {
        set_error("bad cell-residual arguments");
        return SIMM_EINVAL;
    }
    if (mem != SIMM_MEM_HOST && mem != SIMM_MEM_DEVICE) {
        set_error("mem must be SIMM_MEM_HOST or SIMM_MEM_DEVICE");
        return SIMM_EINVAL;
    }
    if (params->gauss_per_edge < 1 || !(params->x1 > params->x0) || params->n1 < 1) {
        set_error("bad region or gauss_per_edge < 1");
        return SIMM_EINVAL;
    }
    if (params->gauss_per_edge > 64) {
        set_error("gauss_per_edge above 64 is not supported");
        return SIMM_EUNSUPPORTED;
    }
    if (n_squares == 0) return SIMM_OK;
    if (!s->H) {
        set_error("shift has no Arnoldi matrix");
        return SIMM_EINVAL;
    }
    SIMM_TRY(check_device());
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    Rule rule;
    SIMM_TRY(rule.make(params->gauss_per_edge, st));
    IndicatorParams ip;
    ip.x0 = params->x0;
    ip.y0 = params->y0;
    ip.w1 = (params->x1 - params->x0) / params->n1;
    ip.eps0 = params->eps0;
    ip.delta0 = params->delta0;
    ip.tau = params->tau;
    DevBuf sq_buf, out_buf;
    const int64_t* sq_dev = squares;
    unsigned long long* out_dev = reinterpret_cast<unsigned long long*>(rho_max);   // doubles >= 0 as bit patterns
    if (mem == SIMM_MEM_HOST) {
        SIMM_TRY(sq_buf.alloc(sizeof(int64_t) * 2 * (size_t)n_squares, st));
        SIMM_TRY(out_buf.alloc(sizeof(double) * (size_t)n_squares, st));
        SIMM_HIP_TRY(hipMemcpyAsync(sq_buf.p, squares, sizeof(int64_t) * 2 * (size_t)n_squares,
                                    hipMemcpyHostToDevice, st));
        sq_dev = sq_buf.as<int64_t>();
        out_dev = out_buf.as<unsigned long long>();
    }
    SIMM_TRY(cells_resid(s->H, s->m + 1, s->m_eff, s->h_last, s->sigma, sq_dev, n_squares, level, ip, rule.dev, out_dev,
                         st));
    if (mem == SIMM_MEM_HOST) {
        SIMM_HIP_TRY(hipMemcpyAsync(rho_max, out_dev, sizeof(double) * (size_t)n_squares, hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));
    }
    return SIMM_OK;
}

simm_status simm_indicators(const simm_shift* shifts, int32_t n_shifts, const int64_t* regions, int64_t n_regions,
                            const simm_params* params, double* indicator, double* rho_max, double* nsf, double* nsc,
                            double* Tf, uint8_t* decision, double* sums, int32_t m_max, int32_t mem,
                            void* hip_stream) {
    clear_error();
    if (!shifts || n_shifts < 1 || (!regions && n_regions > 0) || n_regions < 0 || !params) {
        set_error("bad indicator arguments");
        return SIMM_EINVAL;
    }
    if (mem != SIMM_MEM_HOST && mem != SIMM_MEM_DEVICE) {
        set_error("mem must be SIMM_MEM_HOST or SIMM_MEM_DEVICE");
        return SIMM_EINVAL;
    }
    if (params->gauss_per_edge < 1) {
        set_error("gauss_per_edge >= 1");
        return SIMM_EINVAL;
    }
    if (params->gauss_per_edge > 64) {
        set_error("gauss_per_edge above 64 is not supported");
        return SIMM_EUNSUPPORTED;
    }
    if (!(params->x1 > params->x0) || params->n1 < 1) {
        set_error("bad region");
        return SIMM_EINVAL;
    }
    int mmax = 1;
    for (int s = 0; s < n_shifts; ++s) {
        if (!shifts[s]) return SIMM_EINVAL;
        mmax = std::max(mmax, shifts[s]->m_eff);
    }
    if (sums && m_max < mmax) {
        set_error("m_max smaller than a shift's m_eff");
        return SIMM_EINVAL;
    }
    if (n_regions == 0) return SIMM_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    std::vector<int64_t> regs((size_t)n_regions * 4);
    if (mem == SIMM_MEM_HOST) {
        std::memcpy(regs.data(), regions, sizeof(int64_t) * regs.size());
    } else {
        SIMM_HIP_TRY(hipMemcpyAsync(regs.data(), regions, sizeof(int64_t) * regs.size(), hipMemcpyDeviceToHost, st));
        SIMM_HIP_TRY(hipStreamSynchronize(st));
    }
    for (int64_t r = 0; r < n_regions; ++r) {
        if (regs[4 * r] < 1 || regs[4 * r] > 60 || regs[4 * r + 3] < 0 || regs[4 * r + 3] >= n_shifts) {
            set_error("region row with bad level or shift index");
            return SIMM_EINVAL;
        }
    }
    std::vector<simm_shift_s*> sv(shifts, shifts + n_shifts);
    Rule rule;
    SIMM_TRY(rule.make(params->gauss_per_edge, st));
    DevBuf sb;
    cplx* sums_dev = nullptr;
    if (sums) {
        if (mem == SIMM_MEM_DEVICE) {
            sums_dev = reinterpret_cast<cplx*>(sums);
        } else {
            SIMM_TRY(sb.alloc(sizeof(cplx) * (size_t)n_regions * 2 * m_max, st));
            sums_dev = sb.as<cplx>();
        }
    }
    EvalOut eo;
    SIMM_TRY(evaluate(sv, regs, params, rule, st, eo, sums_dev, sums ? m_max : 0));
    auto put = [&](double* dst, const std::vector<double>& v) -> simm_status {
        if (!dst) return SIMM_OK;
        if (mem == SIMM_MEM_HOST) {
            std::memcpy(dst, v.data(), sizeof(double) * v.size());
        } else {
            SIMM_HIP_TRY(hipMemcpyAsync(dst, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice, st));
        }
        return SIMM_OK;
    };
    SIMM_TRY(put(indicator, eo.indicator));
    SIMM_TRY(put(rho_max, eo.rho));
    SIMM_TRY(put(nsf, eo.nsf));
    SIMM_TRY(put(nsc, eo.nsc));
    SIMM_TRY(put(Tf, eo.Tf));
    if (decision) {
        if (mem == SIMM_MEM_HOST) std::memcpy(decision, eo.decision.data(), eo.decision.size());
        else SIMM_HIP_TRY(hipMemcpyAsync(decision, eo.decision.data(), eo.decision.size(), hipMemcpyHostToDevice, st));
    }
    if (sums && mem == SIMM_MEM_HOST) {
        SIMM_HIP_TRY(hipMemcpyAsync(sums, sums_dev, sizeof(cplx) * (size_t)n_regions * 2 * m_max, hipMemcpyDeviceToHost, st));
    }
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    return SIMM_OK;
}

simm_status simm_gradient(const simm_shift* shifts, int32_t n_shifts, const int64_t* regions, int64_t n_regions,
                          const simm_params* params, int32_t kl1, int32_t ku1, const double* a1_band, double* J,
                          double* dJdp, double* grad_diag, int32_t mem, void* hip_stream) {
    clear_error();
    if (!shifts || n_shifts < 1 || (!regions && n_regions > 0) || n_regions < 0 || !params || !J ||
        (dJdp && (!a1_band || kl1 < 0 || ku1 < 0))) {
        set_error("bad gradient arguments");
        return SIMM_EINVAL;
    }
    if (mem != SIMM_MEM_HOST && mem != SIMM_MEM_DEVICE) {
        set_error("mem must be SIMM_MEM_HOST or SIMM_MEM_DEVICE");
        return SIMM_EINVAL;
    }
    if (params->gauss_per_edge < 1 || params->gauss_per_edge > 64 || !(params->x1 > params->x0) || params->n1 < 1) {
        set_error("bad rule or region (1 <= gauss_per_edge <= 64, x1 > x0, n1 >= 1)");
        return SIMM_EINVAL;
    }
    simm_pencil_s* p = nullptr;
    std::vector<simm_shift_s*> sv(shifts, shifts + n_shifts);
    for (auto* s : sv) {
        if (!s) return SIMM_EINVAL;
        if (p && s->p != p) {
            set_error("the shifts of one gradient call must share one pencil");
            return SIMM_EINVAL;
        }
        p = s->p;
        if (!s->has_factor()) {
            set_error("a shift's factor or Krylov basis was released");
            return SIMM_EINVAL;
        }
        if (s->mixed) {
            set_error("the adjoint gradient needs shifts with an FP64 factor");
            return SIMM_EUNSUPPORTED;
        }
        if (s->m_eff > 128) {
            set_error("Krylov dimension above 128");
            return SIMM_EUNSUPPORTED;
        }
    }
    for (int64_t r = 0; r < n_regions; ++r) {
        if (regions[4 * r] < 1 || regions[4 * r] > 60 || regions[4 * r + 3] < 0 || regions[4 * r + 3] >= n_shifts) {
            set_error("region row with bad level or shift index");
            return SIMM_EINVAL;
        }
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const int64_t n = p->n;
    const cplx* a1 = dJdp ? reinterpret_cast<const cplx*>(a1_band) : nullptr;
    DevBuf a1b, gb;
    if (a1 && mem == SIMM_MEM_HOST) {
        const size_t cnt = (size_t)(kl1 + ku1 + 1) * n;
        if (!finite_c(a1_band, 2 * (int64_t)cnt)) {
            set_error("A1 has NaN/Inf entries");
            return SIMM_EINVAL;
        }
        SIMM_TRY(a1b.alloc(sizeof(cplx) * cnt, st));
        SIMM_HIP_TRY(hipMemcpyAsync(a1b.p, a1_band, sizeof(cplx) * cnt, hipMemcpyHostToDevice, st));
        a1 = a1b.as<cplx>();
    }
    cplx* grad = reinterpret_cast<cplx*>(grad_diag);
    if (grad && mem == SIMM_MEM_HOST) {
        SIMM_TRY(gb.alloc(sizeof(cplx) * (size_t)n, st));
        grad = gb.as<cplx>();
    }
    std::vector<int64_t> regs(regions, regions + 4 * n_regions);
    if (n_regions == 0) {
        *J = 0.0;
        if (dJdp) *dJdp = 0.0;
        if (grad) SIMM_HIP_TRY(hipMemsetAsync(grad, 0, sizeof(cplx) * (size_t)n, st));
    } else {
        SIMM_TRY(gradient(sv, regs, params, kl1, ku1, a1, J, dJdp, grad, st));
    }
    if (grad_diag && mem == SIMM_MEM_HOST)
        SIMM_HIP_TRY(hipMemcpyAsync(grad_diag, grad, sizeof(cplx) * (size_t)n, hipMemcpyDeviceToHost, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    return SIMM_OK;
}

simm_status simm_project(simm_shift s, const double* Y, int64_t c, double* X, double* col_norms, int32_t precision,
                         void* hip_stream) {
    clear_error();
    if (!s || c < 0 || (c > 0 && (!Y || (!X && !col_norms)))) {
        set_error("bad projection arguments");
        return SIMM_EINVAL;
    }
    if (precision != SIMM_PROJ_FP64 && precision != SIMM_PROJ_FP32 && precision != SIMM_PROJ_BF16) {
        set_error("unknown projection precision");
        return SIMM_EINVAL;
    }
    if (!s->has_factor()) {
        set_error("the shift's Krylov basis was released (SIMM_FLAG_RELEASE_FACTORS)");
        return SIMM_EINVAL;
    }
    if (c == 0) return SIMM_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    DevBuf scr;
    const int64_t se = project_scratch_elems(s->p->n, c);
    if (col_norms) SIMM_TRY(scr.alloc(sizeof(double) * (size_t)se, st));
    SIMM_TRY(project(s->p->n, s->m_eff, s->V, s->p->n, reinterpret_cast<const cplx*>(Y), s->m_eff, c,
                     reinterpret_cast<cplx*>(X), col_norms, col_norms ? scr.as<double>() : nullptr, se, precision, st));
    SIMM_HIP_TRY(hipStreamSynchronize(st));
    return SIMM_OK;
}

simm_status simm_project_noalloc(simm_shift s, const double* Y, int64_t c, double* X, double* col_norms,
                                 int32_t precision, void* hip_stream) {
    clear_error();
    if (!s || c < 0 || (c > 0 && (!Y || (!X && !col_norms)))) {
        set_error("bad projection arguments");
        return SIMM_EINVAL;
    }
    if (precision != SIMM_PROJ_FP64 && precision != SIMM_PROJ_FP32 && precision != SIMM_PROJ_BF16) {
        set_error("unknown projection precision");
        return SIMM_EINVAL;
    }
    if (!s->has_factor()) {
        set_error("the shift's Krylov basis was released (SIMM_FLAG_RELEASE_FACTORS)");
        return SIMM_EINVAL;
    }
    if (c == 0) return SIMM_OK;
    const int64_t se = project_scratch_elems(s->p->n, c);
    double* scr = nullptr;
    if (col_norms) {
        if (se > kNoAllocScratchDoubles) {
            char msg[200];
            std::snprintf(msg, sizeof msg,
                          "simm_project_noalloc: the column norms of n = %lld, c = %lld need %lld doubles of scratch, "
                          "more than the %lld the library holds",
                          (long long)s->p->n, (long long)c, (long long)se, (long long)kNoAllocScratchDoubles);
            set_error(msg);
            return SIMM_EUNSUPPORTED;
        }
        SIMM_TRY(noalloc_scratch(&scr));
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    return project(s->p->n, s->m_eff, s->V, s->p->n, reinterpret_cast<const cplx*>(Y), s->m_eff, c,
                   reinterpret_cast<cplx*>(X), col_norms, scr, se, precision, st);
}

simm_status simm_run(simm_pencil p, const simm_params* params, const double* f, int32_t f_mem, void* hip_stream,
                     simm_result* out) {
    clear_error();
    if (!out) return SIMM_EINVAL;
    *out = nullptr;
    if (!p || !f || !params) {
        set_error("bad run arguments");
        return SIMM_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    DevBuf fb;
    const cplx* fd = nullptr;
    SIMM_TRY(to_device_vec(f, f_mem, p->n, fb, &fd, st));
    auto R = std::make_unique<simm_result_s>();
    hipEvent_t e0, e1;
    SIMM_HIP_TRY(hipEventCreate(&e0));
    SIMM_HIP_TRY(hipEventCreate(&e1));
    SIMM_HIP_TRY(hipEventRecord(e0, st));
    simm_status rc;
    {
        // frees during the run (factors computed ahead and dropped, factors released
        // per shift) are collected and done together at its end
        DeferFrees defer(true);
        rc = run(p, params, fd, st, R.get());
    }
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SIMM_OK) return rc;
    R->ms[3] = ms;
    *out = R.release();
    return SIMM_OK;
}

simm_status simm_run_batch(const simm_pencil* pencils, const simm_params* params, const double* const* f,
                           int32_t f_mem, int32_t count, int32_t workers, simm_result* out) {
    clear_error();
    if (!pencils || !params || !f || !out || count < 0 || workers < 1) {
        set_error("bad batch arguments");
        return SIMM_EINVAL;
    }
    for (int32_t i = 0; i < count; ++i) {
        out[i] = nullptr;
        if (!pencils[i] || !f[i]) {
            set_error("null pencil or vector in the batch");
            return SIMM_EINVAL;
        }
    }
    if (count == 0) return SIMM_OK;
    // at most 16 runs in flight: with 24 (and their factors ahead) the HIP runtime ran out
    // of queue resources and aborted a queue (HSA_STATUS_ERROR_OUT_OF_RESOURCES)
    workers = std::min(workers, 16);
    SIMM_TRY(check_device());
    int dev = 0;
    SIMM_HIP_TRY(hipGetDevice(&dev));
    std::vector<BatchItem> items((size_t)count);
    // steps 1-3 of every pencil: runs in flight on streams of their own, each building its
    // shifts one at a time unless asked for more (the runs in flight share the queues)
    std::atomic<int32_t> next{0};
    auto work = [&]() {
        (void)hipSetDevice(dev);
        hipStream_t st = nullptr;
        const hipError_t se = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        for (;;) {
            const int32_t i = next.fetch_add(1);
            if (i >= count) break;
            BatchItem& it = items[(size_t)i];
            it.p = pencils[i];
            it.prm = params[i];
            if (it.prm.lookahead == 0) it.prm.lookahead = 1;
            it.R = std::make_unique<simm_result_s>();
            if (se != hipSuccess) {
                it.rc = SIMM_EHIP;
                it.msg = std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(se);
                continue;
            }
            auto phase = [&]() -> simm_status {
                int nx, ny, K;
                SIMM_TRY(validate_params(&it.prm, it.p->n, &nx, &ny, &K));
                it.R->K = K;
                it.R->prm = it.prm;
                it.R->pencil = it.p;
                DevBuf fb;
                const cplx* fd = nullptr;
                SIMM_TRY(to_device_vec(f[i], f_mem, it.p->n, fb, &fd, st));
                Rule rule;
                SIMM_TRY(rule.make(it.prm.gauss_per_edge, st));
                SIMM_TRY(associate(it.p, &it.prm, fd, st, it.R.get(), rule, nullptr, it.cur));
                SIMM_HIP_TRY(hipStreamSynchronize(st));
                return SIMM_OK;
            };
            const auto t0 = std::chrono::steady_clock::now();
            it.rc = phase();
            if (it.rc != SIMM_OK) it.msg = simm_last_error();
            it.R->ms[3] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (batch_progress())
                std::fprintf(stderr, "[simm batch] pencil %d: n = %lld, %zu shifts, %.0f ms\n", (int)i,
                             (long long)it.p->n, it.R->shifts.size(), it.R->ms[3]);
        }
        if (se == hipSuccess) {
            release_stream_buffers(st);
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    };
    DeferFrees defer(true);
    {
        std::vector<std::thread> pool;
        const int32_t nw = std::min(workers, count);
        for (int32_t w = 0; w < nw; ++w) pool.emplace_back(work);
        for (auto& t : pool) t.join();
    }
    auto fail_at = [&](int32_t i, const std::string& m) {
        set_error("pencil " + std::to_string(i) + ": " + m);
        return items[(size_t)i].rc;
    };
    for (int32_t i = 0; i < count; ++i)
        if (items[(size_t)i].rc != SIMM_OK) return fail_at(i, items[(size_t)i].msg);
    // steps 4-5 of all pencils together, level by level (one stream); pencils whose rule,
    // Krylov dimension, flags or precision differ from the first take the levels one
    // pencil at a time instead
    hipStream_t st = nullptr;
    SIMM_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() {
            release_stream_buffers(s);
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    } guard{st};
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<BatchItem> joint;
    std::vector<int32_t> joint_idx, alone_idx;
    for (int32_t i = 0; i < count; ++i) {
        const simm_params& a = items[0].prm;
        const simm_params& b = items[(size_t)i].prm;
        if (b.m == a.m && b.gauss_per_edge == a.gauss_per_edge && b.flags == a.flags && b.precision == a.precision)
            joint_idx.push_back(i);
        else
            alone_idx.push_back(i);
    }
    {
        std::vector<BatchItem> js;
        for (int32_t i : joint_idx) js.push_back(std::move(items[(size_t)i]));
        simm_status rc = run_batch_levels(js, st);
        for (size_t q = 0; q < joint_idx.size(); ++q) items[(size_t)joint_idx[q]] = std::move(js[q]);
        if (rc != SIMM_OK) return rc;
    }
    for (int32_t i : alone_idx) {
        BatchItem& it = items[(size_t)i];
        Rule rule;
        SIMM_TRY(rule.make(it.prm.gauss_per_edge, st));
        const simm_status rc = level_loop(it.p, &it.prm, st, it.R.get(), rule, nullptr, std::move(it.cur));
        if (rc != SIMM_OK) return fail_at(i, simm_last_error());
    }
    const double levels_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int32_t i = 0; i < count; ++i) {
        BatchItem& it = items[(size_t)i];
        make_clusters(it.R.get());
        const simm_status rc = finish_run(it.R.get(), st);
        if (rc != SIMM_OK) return fail_at(i, simm_last_error());
        it.R->ms[1] += levels_ms;   // the levels of the batch are shared: each run reports the whole
        it.R->ms[3] += levels_ms;
    }
    for (int32_t i = 0; i < count; ++i) out[i] = items[(size_t)i].R.release();
    return SIMM_OK;
}

simm_status simm_batch_tuning(int64_t* entries, int64_t* trials, int32_t* ind_grid, int32_t* proj_grid, int64_t cap) {
    std::lock_guard<std::mutex> lk(g_tune.mu);
    const int64_t ne = (int64_t)(g_tune.ind.size() + g_tune.proj.size());
    if (entries) *entries = ne;
    if (trials) *trials = g_tune.trials;
    int64_t q = 0;
    for (auto& kv : g_tune.ind)
        if (ind_grid && q < cap) ind_grid[q++] = kv.second;
    q = 0;
    for (auto& kv : g_tune.proj)
        if (proj_grid && q < cap) proj_grid[q++] = kv.second;
    return SIMM_OK;
}

simm_status simm_result_summary(simm_result r, int32_t* K, int32_t* n_shifts, int64_t* n_clusters,
                                int64_t* n_unresolved) {
    if (!r) return SIMM_EINVAL;
    if (K) *K = r->K;
    if (n_shifts) *n_shifts = (int32_t)r->shifts.size();
    if (n_clusters) *n_clusters = (int64_t)r->clusters.size();
    if (n_unresolved) {
        int64_t u = 0;
        if (!r->levels.empty())
            for (auto d : r->levels.back().decision) u += (d == SIMM_UNRESOLVED);
        *n_unresolved = u;
    }
    return SIMM_OK;
}

simm_status simm_result_level(simm_result r, int32_t level, int64_t* n_tested, int64_t* ix, int64_t* iy,
                              int32_t* shift, double* indicator, double* rho_max, uint8_t* decision, int64_t cap) {
    clear_error();
    if (!r || !n_tested || level < 1 || level > (int32_t)r->levels.size()) {
        set_error("bad level");
        return SIMM_EINVAL;
    }
    const LevelRec& L = r->levels[level - 1];
    const int64_t N = (int64_t)L.ix.size();
    *n_tested = N;
    if (cap < N) {
        set_error("cap smaller than the number of squares");
        return SIMM_EINVAL;
    }
    for (int64_t q = 0; q < N; ++q) {
        if (ix) ix[q] = L.ix[q];
        if (iy) iy[q] = L.iy[q];
        if (shift) shift[q] = L.shift[q];
        if (indicator) indicator[q] = L.indicator[q];
        if (rho_max) rho_max[q] = L.rho_max[q];
        if (decision) decision[q] = L.decision[q];
    }
    return SIMM_OK;
}

simm_status simm_result_full_indicators(simm_result r, int32_t level, double* out, int64_t cap) {
    clear_error();
    if (!r || level < 1 || level > (int32_t)r->levels.size()) {
        set_error("bad level");
        return SIMM_EINVAL;
    }
    const LevelRec& L = r->levels[level - 1];
    const int64_t N = (int64_t)L.full_indicator.size();
    if (cap < N || (!out && N > 0)) {
        set_error("cap smaller than the number of squares");
        return SIMM_EINVAL;
    }
    for (int64_t q = 0; q < N; ++q) out[q] = L.full_indicator[q];
    return SIMM_OK;
}

simm_status simm_result_shift(simm_result r, int32_t idx, simm_shift* out) {
    if (!r || !out || idx < 0 || idx >= (int32_t)r->shifts.size()) return SIMM_EINVAL;
    *out = r->shifts[idx].get();
    return SIMM_OK;
}

simm_status simm_result_clusters(simm_result r, int64_t* n, double* lam, double* lam_ritz, int32_t* shift,
                                 int32_t* flags, int64_t cap) {
    clear_error();
    if (!r || !n) return SIMM_EINVAL;
    const int64_t N = (int64_t)r->clusters.size();
    *n = N;
    if (cap < N) {
        set_error("cap smaller than the number of clusters");
        return SIMM_EINVAL;
    }
    for (int64_t q = 0; q < N; ++q) {
        const ClusterRec& c = r->clusters[q];
        if (lam) {
            lam[2 * q] = c.lam.re;
            lam[2 * q + 1] = c.lam.im;
        }
        if (lam_ritz) {
            lam_ritz[2 * q] = c.lam_ritz.re;
            lam_ritz[2 * q + 1] = c.lam_ritz.im;
        }
        if (shift) shift[q] = c.shift;
        if (flags) flags[q] = c.flags;
    }
    return SIMM_OK;
}

simm_status simm_multiplicities(simm_result r, const double* F, int32_t k, int32_t f_mem, double rel_tol,
                                void* hip_stream, int32_t* mult, double* sv, int64_t cap) {
    clear_error();
    if (!r || !F || !mult || k < 1 || k > 64 || !(rel_tol > 0.0) || !(rel_tol < 1.0)) {
        set_error("bad multiplicity arguments (need 1 <= k <= 64, 0 < rel_tol < 1)");
        return SIMM_EINVAL;
    }
    if (cap < (int64_t)r->clusters.size()) {
        set_error("cap smaller than the number of clusters");
        return SIMM_EINVAL;
    }
    if (!r->pencil || r->levels.empty()) {
        set_error("result has no levels");
        return SIMM_EINVAL;
    }
    for (const auto& sh : r->shifts)
        if (!sh->has_factor()) {
            set_error("the run's factors were released (SIMM_FLAG_RELEASE_FACTORS)");
            return SIMM_EINVAL;
        }
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    DevBuf fb;
    const cplx* fd = nullptr;
    SIMM_TRY(to_device_vec(F, f_mem, r->pencil->n * (int64_t)k, fb, &fd, st));
    return multiplicities(r, fd, k, rel_tol, st, mult, sv);
}

simm_status simm_result_stats(simm_result r, double* ms4, int64_t* counters3) {
    if (!r) return SIMM_EINVAL;
    if (ms4)
        for (int i = 0; i < 4; ++i) ms4[i] = r->ms[i];
    if (counters3)
        for (int i = 0; i < 3; ++i) counters3[i] = r->counters[i];
    return SIMM_OK;
}

simm_status simm_result_refine_stats(simm_result r, int64_t* solves, int64_t* corrections, int32_t* fallbacks,
                                     double* max_eta) {
    if (!r) return SIMM_EINVAL;
    if (solves) *solves = r->refine_solves;
    if (corrections) *corrections = r->refine_corrections;
    if (fallbacks) *fallbacks = r->refine_fallbacks;
    if (max_eta) *max_eta = r->refine_max_eta;
    return SIMM_OK;
}

simm_status simm_shift_refine_stats(simm_shift s, int64_t* solves, int64_t* corrections, double* max_eta) {
    clear_error();
    if (!s) return SIMM_EINVAL;
    long long stats[2] = {0, 0};
    unsigned long long eta_bits = 0;
    if (s->mixed && s->ref_mem) {
        SIMM_HIP_TRY(hipMemcpy(stats, s->rst.stats, sizeof(stats), hipMemcpyDeviceToHost));
        SIMM_HIP_TRY(hipMemcpy(&eta_bits, s->rst.norms + 3, sizeof(eta_bits), hipMemcpyDeviceToHost));
    }
    double eta = 0.0;
    std::memcpy(&eta, &eta_bits, sizeof(eta));
    if (solves) *solves = stats[0];
    if (corrections) *corrections = stats[1];
    if (max_eta) *max_eta = eta;
    return SIMM_OK;
}

simm_status simm_shift_factor_info(simm_shift s, int64_t* block_len, int32_t* fallback, double* eta) {
    clear_error();
    if (!s) return SIMM_EINVAL;
    if (block_len) *block_len = s->part_bs;
    if (fallback) *fallback = s->part_fallback ? 1 : 0;
    if (eta) *eta = s->part_eta;
    return SIMM_OK;
}

simm_status simm_result_kernel_stats(simm_result r, double* ms, int64_t* launches) {
    if (!r) return SIMM_EINVAL;
    for (int k = 0; k < SIMM_K_COUNT; ++k) {
        if (ms) ms[k] = r->kms[k];
        if (launches) launches[k] = r->kcnt[k];
    }
    return SIMM_OK;
}

void simm_result_destroy(simm_result r) { delete r; }

}  // extern "C"
