// amq_math.h — binary64 helpers shared by the generation and sweep kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace amq {

// p*g + c rounded once (v_fma_f64), with c in a register of its own.  The
// compiler's selection of a polynomial step with a loop-invariant, non-inline
// coefficient is the two-address v_fmac_f64 plus a v_mov_b64 that copies the
// coefficient into the accumulator first: one extra vector instruction per
// step.  The three-address form needs no copy; the result is the same fma.
__device__ __forceinline__ double fma3(double p, double g, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(g), "v"(c));
    return r;
}

// exp(x) in binary64: n = rint(x log2(e)), g = x - n ln 2 (Cody-Waite: ln 2
// split into a 53-bit head and its tail, each product taken exactly inside
// an fma), |g| <= 0.3466; exp(x) = 2^n e^g with e^g from its Taylor series to
// degree 12 (truncation below 0.3466^13 / 13! < 2e-16 relative).  Intended
// for the arguments the kernels produce (|x| < 700); very negative x
// underflows to 0 through ldexp.  kFma3 evaluates the polynomial with fma3
// (same values): it pays where the coefficients stay in vector registers
// across a loop, as in path generation; elsewhere the compiler's own form is
// kept.
// 1/4! and 1/8! one ulp above their nearest binary64 values (7e-18 and 3e-21
// higher, far below either polynomial's truncation): rounded to nearest, each
// shares its low 32 bits with 1/3! or 1/7!, and the compiler then keeps one
// register for both low words and copies it into place inside the loop.
constexpr double kInvFact4 = 0x1.5555555555556p-5, kInvFact8 = 0x1.a01a01a01a01bp-16;

template <bool kFma3 = false>
__device__ __forceinline__ double exp_poly(double x)
{
    const auto step = [](double p, double g, double c) { return kFma3 ? fma3(p, g, c) : fma(p, g, c); };
    const double n = rint(x * 1.4426950408889634);
    const double g = fma(-n, 2.3190468138462996e-17, fma(-n, 0.69314718055994529, x));
    double p = 1.0 / 479001600.0;                  // 1/12!
    p = step(p, g, 1.0 / 39916800.0);               // 1/11!
    p = step(p, g, 1.0 / 3628800.0);
    p = step(p, g, 1.0 / 362880.0);
    p = step(p, g, kInvFact8);
    p = step(p, g, 1.0 / 5040.0);
    p = step(p, g, 1.0 / 720.0);
    p = step(p, g, 1.0 / 120.0);
    p = step(p, g, kInvFact4);
    p = step(p, g, 1.0 / 6.0);
    p = fma(p, g, 0.5);
    p = fma(p, g, 1.0);
    p = fma(p, g, 1.0);
    return ldexp(p, (int)n);
}

// exp(x) to about 1e-10 relative, for values that are then rounded to
// binary32 (0.003 of a binary32 ulp): the same reduction with a degree-8
// Taylor polynomial (truncation below 0.3466^9 / 9! < 2.1e-10).
__device__ __forceinline__ double exp_poly_f32(double x)
{
    const double n = rint(x * 1.4426950408889634);
    const double g = fma(-n, 2.3190468138462996e-17, fma(-n, 0.69314718055994529, x));
    double p = kInvFact8;
    p = fma3(p, g, 1.0 / 5040.0);
    p = fma3(p, g, 1.0 / 720.0);
    p = fma3(p, g, 1.0 / 120.0);
    p = fma3(p, g, kInvFact4);
    p = fma3(p, g, 1.0 / 6.0);
    p = fma(p, g, 0.5);
    p = fma(p, g, 1.0);
    p = fma(p, g, 1.0);
    return ldexp(p, (int)n);
}

// 1/sqrt(d) and 1/d for d > 0 in binary64: hardware estimate refined by
// Newton steps (each roughly doubles the correct bits; two from the ~2^-22
// estimate reach full binary64 precision).
__device__ __forceinline__ double rsqrt_f64(double d)
{
    double y = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    y = y * fma(-hd * y, y, 1.5);
    y = y * fma(-hd * y, y, 1.5);
    return y;
}

__device__ __forceinline__ double rcp_f64(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    y = y * fma(-d, y, 2.0);
    y = y * fma(-d, y, 2.0);
    return y;
}

}  // namespace amq
