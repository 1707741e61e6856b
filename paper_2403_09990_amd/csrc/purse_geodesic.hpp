// One step of the MEGB geodesic descent on unit quaternions (rotation chain)
// or points (translation chain), with the float32 sin/cos and arctangent it
// uses.  Shared by the descent and by its replay in the backward, so both
// take bitwise the same steps.
#pragma once

#include <hip/hip_runtime.h>

namespace purse {

// From this step on the descent moves by at most (pi/2)/16 in quaternion
// angle, where the short sin/cos series below are exact to float32.
constexpr int kShortSeriesStep = 16;

// sin and cos on [0, pi/2] by their Taylor series through x^13 and x^14
// (truncation below 7e-10 there), evaluated in x^2 by Horner's rule.
__device__ __forceinline__ void sincos_quadrant(float x, float &s, float &c) {
  const float z = x * x;
  float ps = 1.f / 6227020800.f;       // 1/13!
  ps = ps * z - 1.f / 39916800.f;      // 1/11!
  ps = ps * z + 1.f / 362880.f;        // 1/9!
  ps = ps * z - 1.f / 5040.f;          // 1/7!
  ps = ps * z + 1.f / 120.f;
  ps = ps * z - 1.f / 6.f;
  s = x + x * (ps * z);
  float pc = 1.f / 87178291200.f;      // 1/14!
  pc = pc * z - 1.f / 479001600.f;     // 1/12!
  pc = pc * z + 1.f / 3628800.f;       // 1/10!
  pc = pc * z - 1.f / 40320.f;         // 1/8!
  pc = pc * z + 1.f / 720.f;
  pc = pc * z - 1.f / 24.f;
  pc = pc * z + 0.5f;
  c = 1.f - pc * z;
}

// sin and cos on [0, pi/32] by their Taylor series through x^7 and x^6
// (truncation below 3e-13 there).
__device__ __forceinline__ void sincos_small(float x, float &s, float &c) {
  const float z = x * x;
  float ps = -1.f / 5040.f;
  ps = ps * z + 1.f / 120.f;
  ps = ps * z - 1.f / 6.f;
  s = x + x * (ps * z);
  float pc = -1.f / 720.f;
  pc = pc * z + 1.f / 24.f;
  pc = pc * z - 0.5f;
  c = 1.f + pc * z;
}

// atan w for 0 <= w <= tan(pi/8): the odd Taylor series through w^19
// (truncation below 5e-10 there).
__device__ __forceinline__ float atan_eighth(float w) {
  const float z = w * w;
  float p = 1.f / 19.f;
  p = p * z - 1.f / 17.f;
  p = p * z + 1.f / 15.f;
  p = p * z - 1.f / 13.f;
  p = p * z + 1.f / 11.f;
  p = p * z - 1.f / 9.f;
  p = p * z + 1.f / 7.f;
  p = p * z - 1.f / 5.f;
  p = p * z + 1.f / 3.f;
  return w - w * (p * z);
}

// C <- C Exp(Log(C^T R_s) / i) (rotation), c <- c + (t_s - c) / i (translation).
// For unit quaternions a (centre) and b (sample, sign chosen so that a.b >= 0)
// at quaternion angle h, the step is the spherical interpolation at 1/i:
//   sin((1 - 1/i) h) / sin h a + sin(h / i) / sin h b
//   = (cos(h/i) - cos h sin(h/i) / sin h) a + sin(h/i) / sin h b.
// The chords |a - b'| = 2 sin(h/2) and |a + b'| = 2 cos(h/2), both formed
// directly, stay accurate for small angles; h/4 = atan(|a - b'| / (2 + |a + b'|))
// (half-angle tangent of h/2), its argument at most tan(pi/8).  b' = a gives
// sin(h/i) = 0 and no move (sin h is clamped away from 0 for that case).
// inv is 1/i, correctly rounded; SMALL (i >= kShortSeriesStep) selects the
// short sin/cos series.
template <bool SMALL>
__device__ __forceinline__ float4 geodesic_step_inv(float4 a, float4 b, float inv, int chain) {
  if (chain == 1) return make_float4(a.x + (b.x - a.x) * inv, a.y + (b.y - a.y) * inv, a.z + (b.z - a.z) * inv, 1.f);
  const float m0 = a.x - b.x, m1 = a.y - b.y, m2 = a.z - b.z, m3 = a.w - b.w;
  const float p0 = a.x + b.x, p1 = a.y + b.y, p2 = a.z + b.z, p3 = a.w + b.w;
  const float x = m0 * m0 + m1 * m1 + m2 * m2 + m3 * m3;  // |a - b|^2
  const float y = p0 * p0 + p1 * p1 + p2 * p2 + p3 * p3;  // |a + b|^2
  const bool flip = x > y;                                // a . b < 0: use b' = -b
  const float xs = flip ? y : x;                          // |a - b'|^2
  const float ys = flip ? x : y;                          // |a + b'|^2
  const float rx = __builtin_amdgcn_sqrtf(xs), ry = __builtin_amdgcn_sqrtf(ys);
  const float quarter = atan_eighth(rx * __builtin_amdgcn_rcpf(2.f + ry));  // h / 4
  float st, ct;
  if (SMALL)
    sincos_small(4.f * quarter * inv, st, ct);            // sin, cos of h / i
  else
    sincos_quadrant(4.f * quarter * inv, st, ct);
  const float sh = 0.5f * rx * ry;                        // sin h
  const float chh = 1.f - 0.5f * xs;                      // cos h
  const float cb = st * __builtin_amdgcn_rcpf(fmaxf(sh, 1e-30f));
  const float ca = ct - chh * cb;
  const float cbs = flip ? -cb : cb;
  float4 q = make_float4(ca * a.x + cbs * b.x, ca * a.y + cbs * b.y, ca * a.z + cbs * b.z, ca * a.w + cbs * b.w);
  const float nn = __builtin_amdgcn_rsqf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);  // |q| ~ 1
  return make_float4(q.x * nn, q.y * nn, q.z * nn, q.w * nn);
}

__device__ __forceinline__ float4 geodesic_step_inv(float4 a, float4 b, float inv, int i, int chain) {
  return i >= kShortSeriesStep ? geodesic_step_inv<true>(a, b, inv, chain) : geodesic_step_inv<false>(a, b, inv, chain);
}

__device__ __forceinline__ float4 geodesic_step(float4 a, float4 b, int i, int chain) {
  return geodesic_step_inv(a, b, 1.f / (float)i, i, chain);
}

}  // namespace purse
