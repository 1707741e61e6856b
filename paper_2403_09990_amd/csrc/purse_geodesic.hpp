// One step of the MEGB geodesic descent on unit quaternions (rotation chain)
// or points (translation chain), with the float32 sin/cos and arctangent it
// uses.  Shared by the descent and by its replay in the backward, so both
// take bitwise the same steps.
#pragma once

#include <hip/hip_runtime.h>

namespace purse {

// v of lane `lane` of the wavefront (a wave-uniform lane index).
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// From this step on the descent moves by at most (pi/2)/16 in quaternion
// angle, where the short sin/cos series below are exact to float32.
constexpr int kShortSeriesStep = 16;

// sin and cos on [0, pi/2] by their Taylor series through x^13 and x^14
// (truncation below 7e-10 there), evaluated in x^2 by Horner's rule.
__device__ __forceinline__ void sincos_quadrant(float x, float &s, float &c) {
  const float z = x * x;
  float ps = 1.f / 6227020800.f;       // 1/13!
  ps = fmaf(ps, z, -1.f / 39916800.f);      // 1/11!
  ps = fmaf(ps, z, 1.f / 362880.f);        // 1/9!
  ps = fmaf(ps, z, -1.f / 5040.f);          // 1/7!
  ps = fmaf(ps, z, 1.f / 120.f);
  ps = fmaf(ps, z, -1.f / 6.f);
  s = fmaf(x, ps * z, x);
  float pc = 1.f / 87178291200.f;      // 1/14!
  pc = fmaf(pc, z, -1.f / 479001600.f);     // 1/12!
  pc = fmaf(pc, z, 1.f / 3628800.f);       // 1/10!
  pc = fmaf(pc, z, -1.f / 40320.f);         // 1/8!
  pc = fmaf(pc, z, 1.f / 720.f);
  pc = fmaf(pc, z, -1.f / 24.f);
  pc = fmaf(pc, z, 0.5f);
  c = fmaf(-pc, z, 1.f);
}

// sin and cos on [0, pi/32] by their Taylor series through x^7 and x^6
// (truncation below 3e-13 there).
__device__ __forceinline__ void sincos_small(float x, float &s, float &c) {
  const float z = x * x;
  float ps = -1.f / 5040.f;
  ps = fmaf(ps, z, 1.f / 120.f);
  ps = fmaf(ps, z, -1.f / 6.f);
  s = fmaf(x, ps * z, x);
  float pc = -1.f / 720.f;
  pc = fmaf(pc, z, 1.f / 24.f);
  pc = fmaf(pc, z, -0.5f);
  c = fmaf(pc, z, 1.f);
}

// atan w for 0 <= w <= tan(pi/8): w + w^3 P(w^2), P of degree 4 fitted to
// (atan w - w) / w^3 by Lawson's iteratively reweighted least squares toward
// the minimax fit (paper_2403_09990_amd/fit_series.py): error below 2e-10
// in exact arithmetic, at the float32 rounding level when evaluated here.
__device__ __forceinline__ float atan_eighth(float w) {
  const float z = w * w;
  float p = -5.945400894e-02f;
  p = fmaf(p, z, 1.053481475e-01f);
  p = fmaf(p, z, -1.423431039e-01f);
  p = fmaf(p, z, 1.999788284e-01f);
  p = fmaf(p, z, -3.333330154e-01f);
  return fmaf(w, p * z, w);
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
// The rotation step in three stages, which geodesic_step_inv composes and
// which a caller may interleave with other work: the chords' lengths from
// x = |a - b|^2 and y = |a + b|^2 ...
struct RotChords {
  float xs, rx, ry;  // |a - b'|^2, |a - b'|, |a + b'|
  bool flip;         // a . b < 0: b' = -b
};
__device__ __forceinline__ RotChords rot_chords(float x, float y) {
  RotChords c;
  c.flip = x > y;
  c.xs = c.flip ? y : x;
  const float ys = c.flip ? x : y;
  c.rx = __builtin_amdgcn_sqrtf(c.xs);
  c.ry = __builtin_amdgcn_sqrtf(ys);
  return c;
}
// ... the angle h / i of the step ...
__device__ __forceinline__ float rot_step_angle(const RotChords &c, float inv) {
  const float quarter = atan_eighth(c.rx * __builtin_amdgcn_rcpf(2.f + c.ry));  // h / 4
  return (4.f * quarter) * inv;
}
// ... and the interpolation itself, renormalised.
template <bool SMALL>
__device__ __forceinline__ float4 rot_interp(const RotChords &c, float th, float4 a, float4 b) {
  float st, ct;
  if (SMALL)
    sincos_small(th, st, ct);  // sin, cos of h / i
  else
    sincos_quadrant(th, st, ct);
  const float sh = (0.5f * c.rx) * c.ry;                  // sin h
  const float chh = fmaf(-0.5f, c.xs, 1.f);               // cos h
  const float cb = st * __builtin_amdgcn_rcpf(fmaxf(sh, 1e-30f));
  const float ca = fmaf(-chh, cb, ct);
  const float cbs = c.flip ? -cb : cb;
  const float4 q = make_float4(fmaf(cbs, b.x, ca * a.x), fmaf(cbs, b.y, ca * a.y), fmaf(cbs, b.z, ca * a.z),
                               fmaf(cbs, b.w, ca * a.w));
  const float nn = __builtin_amdgcn_rsqf(fmaf(q.w, q.w, fmaf(q.z, q.z, fmaf(q.y, q.y, q.x * q.x))));  // |q| ~ 1
  return make_float4(q.x * nn, q.y * nn, q.z * nn, q.w * nn);
}

// |a - b|^2 and |a + b|^2 of two quaternions, formed directly.
__device__ __forceinline__ void rot_chord_sq(float4 a, float4 b, float &x, float &y) {
  const float m0 = a.x - b.x, m1 = a.y - b.y, m2 = a.z - b.z, m3 = a.w - b.w;
  const float p0 = a.x + b.x, p1 = a.y + b.y, p2 = a.z + b.z, p3 = a.w + b.w;
  x = fmaf(m3, m3, fmaf(m2, m2, fmaf(m1, m1, m0 * m0)));
  y = fmaf(p3, p3, fmaf(p2, p2, fmaf(p1, p1, p0 * p0)));
}

template <bool SMALL>
__device__ __forceinline__ float4 geodesic_step_inv(float4 a, float4 b, float inv, int chain) {
  // (explicit fused multiply-adds: every caller rounds the step the same way)
  if (chain == 1) return make_float4(fmaf(b.x - a.x, inv, a.x), fmaf(b.y - a.y, inv, a.y), fmaf(b.z - a.z, inv, a.z), 1.f);
  float x, y;
  rot_chord_sq(a, b, x, y);
  const RotChords c = rot_chords(x, y);
  return rot_interp<SMALL>(c, rot_step_angle(c, inv), a, b);
}

__device__ __forceinline__ float4 geodesic_step_inv(float4 a, float4 b, float inv, int i, int chain) {
  return i >= kShortSeriesStep ? geodesic_step_inv<true>(a, b, inv, chain) : geodesic_step_inv<false>(a, b, inv, chain);
}

__device__ __forceinline__ float4 geodesic_step(float4 a, float4 b, int i, int chain) {
  return geodesic_step_inv(a, b, 1.f / (float)i, i, chain);
}

}  // namespace purse
