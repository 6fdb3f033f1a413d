// Per-pair geometry shared by the pair kernels: e = exp(i k r)/r, 1/r^2 and
// k r for d = x_target - y_source, with the phase reduced in FP64 on both
// precision paths (paper: the midpoint rule applied to the kernels of
// Theorem 3, eq_vsie, with G = exp(i k r)/(4 pi r); the 1/(4 pi) is carried by
// the source weights).
#pragma once

#include <hip/hip_runtime.h>

namespace vsie {
namespace geom {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.1415926535897932384626433832795;

// ---------------------------------------------------------------------------
// FP64 sin and cos of pi g for |g| <= 1/2 (x = pi g in [-pi/2, pi/2]):
// Maclaurin series of sin through x^21 and of cos through x^22; the first
// omitted terms, (pi/2)^23/23! and (pi/2)^24/24!, are below 2e-18.
__device__ __forceinline__ void sincos_halfturn_f64(double g, double &sn, double &cs) {
    const double x = g * kPi;
    const double z = x * x;
    double ps = -1.0 / 51090942171709440000.0;        // -1/21!
    ps = fma(ps, z, 1.0 / 121645100408832000.0);       //  1/19!
    ps = fma(ps, z, -1.0 / 355687428096000.0);         // -1/17!
    ps = fma(ps, z, 1.0 / 1307674368000.0);            //  1/15!
    ps = fma(ps, z, -1.0 / 6227020800.0);              // -1/13!
    ps = fma(ps, z, 1.0 / 39916800.0);                 //  1/11!
    ps = fma(ps, z, -1.0 / 362880.0);                  // -1/9!
    ps = fma(ps, z, 1.0 / 5040.0);                     //  1/7!
    ps = fma(ps, z, -1.0 / 120.0);                     // -1/5!
    ps = fma(ps, z, 1.0 / 6.0);                        //  1/3!
    sn = fma(-ps * z, x, x);
    double pc = 1.0 / 1124000727777607680000.0;        //  1/22!
    pc = fma(pc, z, -1.0 / 2432902008176640000.0);     // -1/20!
    pc = fma(pc, z, 1.0 / 6402373705728000.0);         //  1/18!
    pc = fma(pc, z, -1.0 / 20922789888000.0);          // -1/16!
    pc = fma(pc, z, 1.0 / 87178291200.0);              //  1/14!
    pc = fma(pc, z, -1.0 / 479001600.0);               // -1/12!
    pc = fma(pc, z, 1.0 / 3628800.0);                  //  1/10!
    pc = fma(pc, z, -1.0 / 40320.0);                   // -1/8!
    pc = fma(pc, z, 1.0 / 720.0);                      //  1/6!
    pc = fma(pc, z, -1.0 / 24.0);                      // -1/4!
    pc = fma(pc, z, 0.5);                              //  1/2!
    cs = fma(-pc, z, 1.0);
}

// Flip the sign of v when the integer-valued double q is odd.
__device__ __forceinline__ double flip_if_odd(double v, double q) {
    const int qi = static_cast<int>(q);
    return __longlong_as_double(__double_as_longlong(v) ^ (static_cast<long long>(qi & 1) << 63));
}

// Geometry of one pair in FP64: e = exp(i k r)/r, ir2 = 1/r^2 and k r.
// The phase is carried in half turns u = k r / pi = q + g with q = rint(u):
// exp(i pi u) = (-1)^q exp(i pi g), and the sign (-1)^q is folded into 1/r.
// 1/sqrt(r^2): v_rsq_f64 (max relative error 5e-8 measured) and one Newton
// step (error below 3e-15).  MASK selects zero for the pair r = 0.
template <bool MASK>
__device__ __forceinline__ void geom_f64(double dx, double dy, double dz, double k, double khalf,
                                         double &er, double &ei, double &ir2, double &kr) {
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2 * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    if (MASK) y = (r2 > 0.0) ? y : 0.0;
    const double r = r2 * y;
    const double u = r * khalf;
    const double q = rint(u);
    double sn, cs;
    sincos_halfturn_f64(u - q, sn, cs);
    const double ys = flip_if_odd(y, q);
    er = cs * ys;
    ei = sn * ys;
    ir2 = y * y;
    kr = k * r;
}

// Geometry of one pair for the FP32 operator: FP64 coordinate differences and
// phase reduction, FP32 amplitude and trigonometric functions.  r is formed
// from an FP32 reciprocal square root and one FP64 Newton correction, which
// is accurate to ~1e-14 relative: enough to keep the phase error far below
// the FP32 rounding of everything else.  The phase in turns is reduced with
// v_fract_f64 (exact) before it is rounded to FP32.
template <bool MASK>
__device__ __forceinline__ void geom_f32(double dx, double dy, double dz, float k, double kr2pi,
                                         float &er, float &ei, float &ir2, float &kr) {
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const float r2f = static_cast<float>(r2);
    float yf = __builtin_amdgcn_rsqf(r2f);
    if (MASK) yf = (r2 > 0.0) ? yf : 0.0f;
    const float rf = r2f * yf;
    const double rd = static_cast<double>(rf);
    const double e = fma(-rd, rd, r2);
    const double r = fma(e, static_cast<double>(0.5f * yf), rd);
    const float f = static_cast<float>(__builtin_amdgcn_fract(r * kr2pi));
    // v_sin_f32 / v_cos_f32 take their argument in turns
    const float sn = __builtin_amdgcn_sinf(f);
    const float cs = __builtin_amdgcn_cosf(f);
    er = cs * yf;
    ei = sn * yf;
    ir2 = yf * yf;
    kr = k * rf;
}

}  // namespace geom
}  // namespace vsie
