// Device math helpers: sin and cos of the Hubbard-field phases.
//
// FP64: Cody-Waite argument reduction x = k (pi/2) + r, |r| <= pi/4, with pi/2 split
// into three parts whose leading parts have trailing zero bits (so k * part is exact
// for the |x| bound below), followed by the Taylor series of sin and cos truncated
// where the remainder drops below half an ulp on [-pi/4, pi/4].  Arguments outside the
// bound (and NaN/Inf) take the library routine.
#pragma once

#include <hip/hip_runtime.h>

namespace hub {

__device__ __forceinline__ void phase_sincos(double x, double* s, double* c) {
    if (!(fabs(x) < 1.0e5)) {
        sincos(x, s, c);
        return;
    }
    const double k = rint(x * 0.6366197723675814);            // 2/pi
    double r = fma(-k, 0x1.921fb54400000p+0, x);               // pi/2 = P1 + P2 + P3
    r = fma(-k, 0x1.0b4611a600000p-34, r);
    r = fma(-k, 0x1.3198a2e037073p-69, r);
    const double z = r * r;
    // sin r = r + r z Q(z),  Q = -1/3! + z/5! - z^2/7! + ... + z^7/17!
    double qs = 1.0 / 355687428096000.0;                       //  1/17!
    qs = fma(qs, z, -1.0 / 1307674368000.0);                   // -1/15!
    qs = fma(qs, z, 1.0 / 6227020800.0);                       //  1/13!
    qs = fma(qs, z, -1.0 / 39916800.0);                        // -1/11!
    qs = fma(qs, z, 1.0 / 362880.0);                           //  1/9!
    qs = fma(qs, z, -1.0 / 5040.0);                            // -1/7!
    qs = fma(qs, z, 1.0 / 120.0);                              //  1/5!
    qs = fma(qs, z, -1.0 / 6.0);                               // -1/3!
    const double sr = fma(r * z, qs, r);
    // cos r = 1 + z P(z),  P = -1/2! + z/4! - ... - z^8/18!
    double pc = -1.0 / 6402373705728000.0;                     // -1/18!
    pc = fma(pc, z, 1.0 / 20922789888000.0);                   //  1/16!
    pc = fma(pc, z, -1.0 / 87178291200.0);                     // -1/14!
    pc = fma(pc, z, 1.0 / 479001600.0);                        //  1/12!
    pc = fma(pc, z, -1.0 / 3628800.0);                         // -1/10!
    pc = fma(pc, z, 1.0 / 40320.0);                            //  1/8!
    pc = fma(pc, z, -1.0 / 720.0);                             // -1/6!
    pc = fma(pc, z, 1.0 / 24.0);                               //  1/4!
    pc = fma(pc, z, -0.5);                                     // -1/2!
    const double cr = fma(pc, z, 1.0);
    const int q = (int)k & 3;
    const double ss = (q & 1) ? cr : sr;
    const double cc = (q & 1) ? sr : cr;
    *s = (q & 2) ? -ss : ss;
    *c = ((q + 1) & 2) ? -cc : cc;
}

// FP32 phases for the single-precision operators: the argument is reduced to at most
// half a revolution (one product, a rounding and an fma) and the CDNA transcendental
// units evaluate sin(2 pi f) and cos(2 pi f).  Accurate to a few ulp of the FP32
// operator's inputs, which is all the single-precision path needs.
__device__ __forceinline__ void phase_sincos_fast(float x, float* s, float* c) {
    if (!(fabsf(x) < 6000.0f)) {
        sincosf(x, s, c);
        return;
    }
    constexpr float kInv2Pi = 0.15915494309189535f;
    const float f = fmaf(x, kInv2Pi, -rintf(x * kInv2Pi));   // revolutions, |f| <= 1/2
    *s = __builtin_amdgcn_sinf(f);
    *c = __builtin_amdgcn_cosf(f);
}

}  // namespace hub
