// Per-pair arithmetic shared by the force kernels: the FP64 r^-3 factor, the
// split form's one-Newton-step factor, and Kahan's compensated addition.
#pragma once

#include <hip/hip_runtime.h>

namespace nb {
namespace pm {

// G m r^-3 to full FP64 accuracy.  The hardware FP64 reciprocal square root
// y0 = v_rsq_f64(r2) has a relative error below 2^-24 (measured 2^-24.2), so
// e = 1 - r2 y0^2 (one FMA; the rounding of y0^2 adds at most 2^-53) is below
// 2^-23, and
//   r^-3 = y0^3 (1 - e)^(-3/2) = y0^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)),
// where the dropped e^3 term is below 1e-20 relative.  (Seeding from the FP32
// v_rsq_f32 instead makes y0^2 exact but needs two conversions, which cost
// more than the slower FP64 transcendental in this loop.)
// c.a = 15/8 and c.b = 3/2 live in vector registers (see vreg_const) so that
// the polynomial is a single v_fma_f64.
struct PolyConst {
    double a, b;
};

static __device__ __forceinline__ double gm_rinv3_f64(double r2, double gm, const PolyConst& c)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double y2 = y * y;
    const double e = __builtin_fma(-r2, y2, 1.0);
    const double g = gm * (y2 * y);
    const double q = e * __builtin_fma(e, c.a, c.b);
    return __builtin_fma(g, q, g);
}

// A loop-invariant constant kept in a vector register: gfx9 VOP3 encodings
// take no literal operand and at most one scalar register, so a polynomial
// with two non-inline constants otherwise costs two extra moves per use.
static __device__ __forceinline__ double vreg_const(double c)
{
    asm volatile("" : "+v"(c));
    return c;
}

// G m r^-3 with one Newton step on the FP32 reciprocal square root:
// y1 = y0 (1 + e/2), e = 1 - r2 y0^2, relative error about 3/2 e^2 (<= 3e-13).
static __device__ __forceinline__ double gm_rinv3_newton1(double r2, double gm)
{
    const double y = (double)__builtin_amdgcn_rsqf((float)r2);
    const double e = __builtin_fma(-r2, y * y, 1.0);
    const double y1 = __builtin_fma(0.5 * y, e, y);
    return gm * (y1 * y1 * y1);
}

// 1/r to full FP64 accuracy (as gm_rinv3_f64): y0 = v_rsq_f64(r2), e = 1 - r2 y0^2,
// 1/r = y0 (1 - e)^(-1/2) = y0 (1 + e/2 + 3/8 e^2 + O(e^3)).
static __device__ __forceinline__ double rinv_f64(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2, y * y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

// Kahan's compensated addition: s + x with the rounding error carried in c.
static __device__ __forceinline__ void kahan_add(float& s, float& c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

}  // namespace pm
}  // namespace nb
