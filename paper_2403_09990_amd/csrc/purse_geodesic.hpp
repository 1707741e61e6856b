// One step of the MEGB geodesic descent on unit quaternions (rotation chain)
// or points (translation chain), with the float32 sin/cos and atan2 it uses.
// Shared by the descent and by its replay in the backward.
#pragma once

#include <hip/hip_runtime.h>

namespace purse {

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

// atan2(y, x) for y, x >= 0 (not both 0): t = min/max in [0, 1]; above
// tan(pi/8) the tangent addition formula gives atan t = pi/4 + atan u with
// u = (t - 1) / (t + 1), so |u| <= tan(pi/8); the odd Taylor series of atan u
// through u^19 (truncation below 5e-10) follows; y > x reflects about pi/4.
__device__ __forceinline__ float atan2_quadrant(float y, float x) {
  const float mx = fmaxf(x, y), mn = fminf(x, y);
  const float t = mn * __builtin_amdgcn_rcpf(mx);
  const bool hi = t > 0.41421356f;
  const float u = hi ? (t - 1.f) * __builtin_amdgcn_rcpf(t + 1.f) : t;
  const float z = u * u;
  float p = 1.f / 19.f;
  p = p * z - 1.f / 17.f;
  p = p * z + 1.f / 15.f;
  p = p * z - 1.f / 13.f;
  p = p * z + 1.f / 11.f;
  p = p * z - 1.f / 9.f;
  p = p * z + 1.f / 7.f;
  p = p * z - 1.f / 5.f;
  p = p * z + 1.f / 3.f;
  float a = u - u * (p * z);
  if (hi) a += 0.78539816f;
  return y > x ? 1.57079633f - a : a;
}

// C <- C Exp(Log(C^T R_s) / i) (rotation), c <- c + (t_s - c) / i (translation).
// For unit quaternions a (centre) and b (sample, sign chosen so that a.b >= 0)
// at quaternion angle h, the step is the spherical interpolation at 1/i:
//   sin((1 - 1/i) h) / sin h a + sin(h / i) / sin h b.
// h comes from the chords, sin(h/2) = |a - b'| / 2 and cos(h/2) = |a + b'| / 2,
// both formed directly, which stay accurate for small angles.
__device__ __forceinline__ float4 geodesic_step(float4 a, float4 b, int i, int chain) {
  const float inv = 1.f / (float)i;
  if (chain == 1) return make_float4(a.x + (b.x - a.x) * inv, a.y + (b.y - a.y) * inv, a.z + (b.z - a.z) * inv, 1.f);
  const float m0 = a.x - b.x, m1 = a.y - b.y, m2 = a.z - b.z, m3 = a.w - b.w;
  const float p0 = a.x + b.x, p1 = a.y + b.y, p2 = a.z + b.z, p3 = a.w + b.w;
  const float x = m0 * m0 + m1 * m1 + m2 * m2 + m3 * m3;  // |a - b|^2
  const float y = p0 * p0 + p1 * p1 + p2 * p2 + p3 * p3;  // |a + b|^2
  const bool flip = x > y;                                // a . b < 0: use b' = -b
  const float xs = flip ? y : x;                          // |a - b'|^2
  const float ys = flip ? x : y;                          // |a + b'|^2
  if (!(xs > 0.f)) return a;
  const float half = atan2_quadrant(__builtin_amdgcn_sqrtf(xs), __builtin_amdgcn_sqrtf(ys));  // h / 2
  float st, ct;
  sincos_quadrant(2.f * half * inv, st, ct);              // sin, cos of h / i
  const float sh = 0.5f * __builtin_amdgcn_sqrtf(xs * ys);  // sin h
  const float chh = 1.f - 0.5f * xs;                      // cos h
  const float cb = st * __builtin_amdgcn_rcpf(sh);
  const float ca = ct - chh * cb;
  const float cbs = flip ? -cb : cb;
  float4 q = make_float4(ca * a.x + cbs * b.x, ca * a.y + cbs * b.y, ca * a.z + cbs * b.z, ca * a.w + cbs * b.w);
  const float nn = rsqrtf(q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  return make_float4(q.x * nn, q.y * nn, q.z * nn, q.w * nn);
}

}  // namespace purse
