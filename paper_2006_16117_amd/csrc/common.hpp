// Shared device/host helpers of the SIM-M HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "simm.h"

namespace simm {

// ---------------------------------------------------------------------------
// complex<double> as two interleaved doubles
// ---------------------------------------------------------------------------
struct cplx {
    double re, im;
};

__host__ __device__ inline cplx mk(double r, double i) { return cplx{r, i}; }
__host__ __device__ inline cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplx operator-(cplx a) { return cplx{-a.re, -a.im}; }
__host__ __device__ inline cplx operator*(cplx a, cplx b) {
    return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
__host__ __device__ inline cplx conj(cplx a) { return cplx{a.re, -a.im}; }
__host__ __device__ inline double norm2(cplx a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }
__host__ __device__ inline double cabs(cplx a) { return hypot(a.re, a.im); }
// a - b * c  (fused form used in the sweeps and eliminations)
__host__ __device__ inline cplx fms(cplx a, cplx b, cplx c) {
    return cplx{a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re};
}
// a + b * c
__host__ __device__ inline cplx fma_c(cplx a, cplx b, cplx c) {
    return cplx{a.re + b.re * c.re - b.im * c.im, a.im + b.re * c.im + b.im * c.re};
}
// a + conj(b) * c
__host__ __device__ inline cplx fma_cj(cplx a, cplx b, cplx c) {
    return cplx{a.re + b.re * c.re + b.im * c.im, a.im + b.re * c.im - b.im * c.re};
}
// c ? a : b, component-wise (a struct-valued ?: can be lowered through scratch memory)
__host__ __device__ inline cplx csel(bool c, cplx a, cplx b) { return cplx{c ? a.re : b.re, c ? a.im : b.im}; }

// complex<float>: the storage and arithmetic of the FP32 band factor (same operations)
struct cplxf {
    float re, im;
};
__host__ __device__ inline cplxf operator+(cplxf a, cplxf b) { return cplxf{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cplxf operator-(cplxf a, cplxf b) { return cplxf{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cplxf operator*(cplxf a, cplxf b) {
    return cplxf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline float cabs1(cplxf a) { return fabsf(a.re) + fabsf(a.im); }
__host__ __device__ inline cplxf fms(cplxf a, cplxf b, cplxf c) {
    return cplxf{a.re - b.re * c.re + b.im * c.im, a.im - b.re * c.im - b.im * c.re};
}
__host__ __device__ inline cplxf csel(bool c, cplxf a, cplxf b) { return cplxf{c ? a.re : b.re, c ? a.im : b.im}; }
// widening / rounding between the two
__host__ __device__ inline cplx widen(cplx a) { return a; }
__host__ __device__ inline cplx widen(cplxf a) { return cplx{(double)a.re, (double)a.im}; }
template <typename C>
__host__ __device__ inline C narrow(cplx a);
template <>
__host__ __device__ inline cplx narrow<cplx>(cplx a) { return a; }
template <>
__host__ __device__ inline cplxf narrow<cplxf>(cplx a) { return cplxf{(float)a.re, (float)a.im}; }
// a / b, scaled to avoid overflow (Smith's method)
__host__ __device__ inline cplx cdiv(cplx a, cplx b) {
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return cplx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    } else {
        double r = b.re / b.im, d = b.im + b.re * r;
        return cplx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
    }
}

// ---------------------------------------------------------------------------
// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// and meets the other waves, without waiting on outstanding global loads (a
// plain __syncthreads() also drains every global load in flight, which defeats
// register prefetching in latency-bound loops).  The "memory" clobber keeps the
// compiler from moving memory accesses across it.
// ---------------------------------------------------------------------------
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ---------------------------------------------------------------------------
// error reporting (thread-local message behind simm_last_error)
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
void clear_error();

#define SIMM_HIP_TRY(expr)                                                                  \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess) {                                                             \
            ::simm::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));           \
            return (_e == hipErrorOutOfMemory) ? SIMM_ENOMEM : SIMM_EHIP;                   \
        }                                                                                   \
    } while (0)

// internal status of work given up on purpose (a factor computed ahead that is no
// longer needed); never returned through the C ABI
constexpr simm_status SIMM_ECANCELED = static_cast<simm_status>(7);

#define SIMM_TRY(expr)                         \
    do {                                       \
        simm_status _s = (expr);               \
        if (_s != SIMM_OK) return _s;          \
    } while (0)

}  // namespace simm
