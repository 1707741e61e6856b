// Device-side building blocks of the PURSE sampler and MEGB kernels (gfx950).
//
// Everything here is per-lane register arithmetic: one trajectory (or one
// candidate) per lane, 3x3 algebra unrolled into VGPRs, no shared state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "purse_dual.hpp"
#include "purse_layout.hpp"

namespace purse {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128-bit
// multiplies, a word permutation and a key xor, Weyl key bump between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
    uint64_t hi0 = __umul64hi(m0, c[0]), lo0 = m0 * c[0];
    uint64_t hi1 = __umul64hi(m1, c[2]), lo1 = m1 * c[2];
    uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// ---------------------------------------------------------------------------
// precision-generic scalar helpers (overloads per precision; the float64
// ones are also host functions, so the host tests run the float64 paths)
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
__host__ __device__ inline double dsqrt(double x) { return sqrt(x); }
// the hardware reciprocal square root: for normal inputs it is what rsqrtf
// returns, without rsqrtf's rescaling of denormal inputs.  Every use here
// bounds its input away from the denormal range, discards the result there,
// or (a denormal Cholesky pivot, a rank-one polar input) fails the step
// either way.
__device__ __forceinline__ float drsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__host__ __device__ inline double drsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ void dsincos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void dsincos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float datan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double datan2(double y, double x) { return atan2(y, x); }

// reciprocal: the hardware approximation (1 ulp) in float32, exact otherwise
__device__ __forceinline__ float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ __device__ inline double drcp(double x) { return 1.0 / x; }

// the same functions on dual numbers (value, derivative)
template <typename T> __device__ __forceinline__ Dual<T> drcp(Dual<T> x) {
  T r = drcp(x.v);
  return {r, -x.d * r * r};
}
template <typename T> __device__ __forceinline__ Dual<T> dsqrt(Dual<T> x) {
  T s = dsqrt(x.v);
  return {s, x.d / (T(2) * s)};
}
template <typename T> __device__ __forceinline__ Dual<T> drsqrt(Dual<T> x) {
  T r = drsqrt(x.v);
  return {r, T(-0.5) * r * r * r * x.d};
}
template <typename T> __device__ __forceinline__ void dsincos(Dual<T> x, Dual<T> *s, Dual<T> *c) {
  T sv, cv;
  dsincos(x.v, &sv, &cv);
  *s = Dual<T>(sv, cv * x.d);
  *c = Dual<T>(cv, -sv * x.d);
}
template <typename T> __device__ __forceinline__ Dual<T> datan2(Dual<T> y, Dual<T> x) {
  T den = x.v * x.v + y.v * y.v;
  return {datan2(y.v, x.v), (x.v * y.d - y.v * x.d) / den};
}

// ---------------------------------------------------------------------------
// 3x3 matrices, row-major arrays of 9.
template <typename T>
__device__ __forceinline__ void matmul3(const T A[9], const T B[9], T C[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

template <typename T>
__device__ __forceinline__ void matvec3(const T A[9], const T x[3], T y[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) y[r] = A[3 * r] * x[0] + A[3 * r + 1] * x[1] + A[3 * r + 2] * x[2];
}

template <typename T>
__device__ __forceinline__ void cross3(const T a[3], const T b[3], T c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Coefficients of Exp on so(3): A = sin th / th, B = (1 - cos th) / th^2,
// C = cos th, from th^2.  In general 1 - cos th is written as 2 sin^2(th/2) so
// small angles keep full precision.  In float32 (and its dual numbers), angles
// up to pi/2 use the Taylor series of A, B and C in th^2 instead (through
// th^12, th^12 and th^14: truncation below 5e-10 there), which needs no square
// root or trigonometric call.
template <typename T>
__device__ __forceinline__ void exp_coeffs(T th2, T &A, T &B, T &C) {
  if (th2 < T(1e-12)) {
    A = T(1) - th2 / T(6);
    B = T(0.5) - th2 / T(24);
    C = T(1) - T(0.5) * th2;
  } else {
    T ith = drsqrt(th2);
    T s, c;
    dsincos(T(0.5) * th2 * ith, &s, &c);
    A = T(2) * s * c * ith;
    B = T(2) * s * s * ith * ith;
    C = T(1) - T(2) * s * s;
  }
}

template <typename T>
__device__ __forceinline__ void exp_coeffs_series(T z, T &A, T &B, T &C) {
  A = T(1.f / 6227020800.f);
  A = A * z - 1.f / 39916800.f;
  A = A * z + 1.f / 362880.f;
  A = A * z - 1.f / 5040.f;
  A = A * z + 1.f / 120.f;
  A = A * z - 1.f / 6.f;
  A = A * z + 1.f;
  B = T(1.f / 87178291200.f);
  B = B * z - 1.f / 479001600.f;
  B = B * z + 1.f / 3628800.f;
  B = B * z - 1.f / 40320.f;
  B = B * z + 1.f / 720.f;
  B = B * z - 1.f / 24.f;
  B = B * z + 0.5f;
  C = T(-1.f / 87178291200.f);
  C = C * z + 1.f / 479001600.f;
  C = C * z - 1.f / 3628800.f;
  C = C * z + 1.f / 40320.f;
  C = C * z - 1.f / 720.f;
  C = C * z + 1.f / 24.f;
  C = C * z - 0.5f;
  C = C * z + 1.f;
}

constexpr float kExpSeriesMax = 2.4674011f;  // (pi/2)^2

__device__ __forceinline__ void exp_coeffs(float th2, float &A, float &B, float &C) {
  if (th2 <= kExpSeriesMax) {
    exp_coeffs_series<float>(th2, A, B, C);
  } else {
    float ith = rsqrtf(th2), s, c;
    sincosf(0.5f * th2 * ith, &s, &c);
    A = 2.f * s * c * ith;
    B = 2.f * s * s * ith * ith;
    C = 1.f - 2.f * s * s;
  }
}

__device__ __forceinline__ void exp_coeffs(Dual<float> th2, Dual<float> &A, Dual<float> &B, Dual<float> &C) {
  if (th2.v <= kExpSeriesMax) {
    exp_coeffs_series<Dual<float>>(th2, A, B, C);
  } else {
    Dual<float> ith = drsqrt(th2), s, c;
    dsincos(Dual<float>(0.5f) * th2 * ith, &s, &c);
    A = Dual<float>(2.f) * s * c * ith;
    B = Dual<float>(2.f) * s * s * ith * ith;
    C = Dual<float>(1.f) - Dual<float>(2.f) * s * s;
  }
}

// Exp of so(3): (cos th) I + (sin th / th) [w]x + ((1 - cos th)/th^2) w w^T.
template <typename T>
__device__ __forceinline__ void exp_so3(const T w[3], T R[9]) {
  T th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  T A, B, C;
  exp_coeffs(th2, A, B, C);
  R[0] = C + B * w[0] * w[0];
  R[4] = C + B * w[1] * w[1];
  R[8] = C + B * w[2] * w[2];
  R[1] = B * w[0] * w[1] - A * w[2];
  R[3] = B * w[0] * w[1] + A * w[2];
  R[2] = B * w[0] * w[2] + A * w[1];
  R[6] = B * w[0] * w[2] - A * w[1];
  R[5] = B * w[1] * w[2] - A * w[0];
  R[7] = B * w[1] * w[2] + A * w[0];
}

// Log of SO(3) for angles below pi: th = atan2(|s|, (tr R - 1)/2) with
// s = vee((R - R^T)/2) = sin(th) * axis; returns th * axis.
template <typename T>
__device__ __forceinline__ void log_so3(const T R[9], T w[3]) {
  T s0 = T(0.5) * (R[7] - R[5]), s1 = T(0.5) * (R[2] - R[6]), s2 = T(0.5) * (R[3] - R[1]);
  T c = T(0.5) * (R[0] + R[4] + R[8] - T(1));
  T sn2 = s0 * s0 + s1 * s1 + s2 * s2;
  T f;
  if (sn2 < T(1e-30)) {
    f = T(1);
  } else {
    T isn = drsqrt(sn2);
    f = datan2(sn2 * isn, c) * isn;
  }
  w[0] = f * s0;
  w[1] = f * s1;
  w[2] = f * s2;
}

template <typename T> __host__ __device__ inline bool is_zero(T x) { return x == T(0); }
template <typename T> __device__ __forceinline__ bool is_zero(Dual<T> x) { return x.v == T(0) && x.d == T(0); }

// Rotation in the (p, q) plane that zeroes S[p][q]: t = tan(phi) is the root of
// t^2 + 2 t theta - 1 = 0 of smaller magnitude, theta = (aqq - app) / (2 apq),
// written as t = 2 apq / (dl + sgn(dl) sqrt(dl^2 + 4 apq^2)), dl = aqq - app.
// This form has no 1/apq, so it stays finite (and so do its derivatives) as
// apq -> 0 in the sweeps after convergence.
template <typename T>
__host__ __device__ inline void jacobi_rotate(T S[9], T V[9], int p, int q) {
  T apq = S[3 * p + q];
  if (is_zero(apq)) return;
  T app = S[3 * p + p], aqq = S[3 * q + q];
  T dl = aqq - app;
  T rt = dsqrt(dl * dl + T(4) * apq * apq);
  T den = dl < T(0) ? dl - rt : dl + rt;
  // Equal diagonal entries (dl = 0) with apq^2 below the smallest normal
  // number leave den = 0 (a 0 * inf in tt, and NaN eigenvectors): the root
  // is then tan(pi/4) with the sign of apq.  Equal entries are what a
  // degenerate pair of eigenvalues gives, e.g. M^T M for the sum of
  // rotations about one axis (the MEGB's last iterates when its winners
  // alternate between two samples), once the sweeps have driven apq to
  // underflow.
  T tt = value_of(den) == 0 ? (value_of(apq) > 0 ? T(1) : T(-1)) : T(2) * apq * drcp(den);
  T c = drsqrt(tt * tt + T(1));
  T s = tt * c;
  S[3 * p + p] = app - tt * apq;
  S[3 * q + q] = aqq + tt * apq;
  S[3 * p + q] = T(0);
  S[3 * q + p] = T(0);
  int r = 3 - p - q;
  T arp = S[3 * r + p], arq = S[3 * r + q];
  T nrp = c * arp - s * arq, nrq = s * arp + c * arq;
  S[3 * r + p] = nrp;
  S[3 * p + r] = nrp;
  S[3 * r + q] = nrq;
  S[3 * q + r] = nrq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T vkp = V[3 * k + p], vkq = V[3 * k + q];
    V[3 * k + p] = c * vkp - s * vkq;
    V[3 * k + q] = s * vkp + c * vkq;
  }
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix S (row-major,
// overwritten by its near-diagonal form); V accumulates the eigenvectors as
// columns.
template <typename T>
__host__ __device__ inline void jacobi3(T S[9], T V[9], int sweeps) {
#pragma unroll
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? T(1) : T(0);
  for (int sw = 0; sw < sweeps; ++sw) {
    jacobi_rotate(S, V, 0, 1);
    jacobi_rotate(S, V, 0, 2);
    jacobi_rotate(S, V, 1, 2);
  }
}

template <typename T>
__device__ __forceinline__ void swap_col(T V[9], T lam[3], int a, int b) {
  T t = lam[a];
  lam[a] = lam[b];
  lam[b] = t;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T x = V[3 * k + a];
    V[3 * k + a] = V[3 * k + b];
    V[3 * k + b] = x;
  }
}

// One Newton step of max tr(R^T M) over R = R0 Exp(w): with Y = R0^T M,
// gradient g = vee(Y - Y^T), Hessian tr(Y) I - (Y + Y^T)/2; R <- R0 Exp(H^-1 g).
// Its error scales with the conditioning of the polar factor itself,
// 1 / (s2 + s3), instead of the squared conditioning of the eigenvector route.
template <typename T>
__device__ __forceinline__ void polar_newton(const T M[9], T R[9]) {
  T Y[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[3 * r + c] = R[r] * M[c] + R[3 + r] * M[3 + c] + R[6 + r] * M[6 + c];
  T g[3] = {Y[7] - Y[5], Y[2] - Y[6], Y[3] - Y[1]};
  T tr = Y[0] + Y[4] + Y[8];
  T h00 = tr - Y[0], h11 = tr - Y[4], h22 = tr - Y[8];
  T h01 = T(-0.5) * (Y[1] + Y[3]), h02 = T(-0.5) * (Y[2] + Y[6]), h12 = T(-0.5) * (Y[5] + Y[7]);
  T a00 = h11 * h22 - h12 * h12, a01 = h02 * h12 - h01 * h22, a02 = h01 * h12 - h02 * h11;
  T a11 = h00 * h22 - h02 * h02, a12 = h01 * h02 - h00 * h12, a22 = h00 * h11 - h01 * h01;
  T det = h00 * a00 + h01 * a01 + h02 * a02;
  if (!(det > T(0)) || !(h00 > T(0))) return;
  T id = T(1) / det;
  T w[3] = {(a00 * g[0] + a01 * g[1] + a02 * g[2]) * id, (a01 * g[0] + a11 * g[1] + a12 * g[2]) * id,
            (a02 * g[0] + a12 * g[1] + a22 * g[2]) * id};
  T E[9], Rn[9];
  exp_so3(w, E);
  matmul3(R, E, Rn);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = Rn[k];
}

// Nearest rotation proj_SO3(M) = U diag(1, 1, det(U V^T)) V^T for M = U S V^T.
// From the eigenvectors v1, v2 of M^T M (largest two), u1 = M v1 / |.|,
// u2 = Gram-Schmidt of M v2, u3 = u1 x u2, v3 = v1 x v2; R = sum u_k v_k^T.
// One Newton step polishes the result.
// Returns false when the step is ill-conditioned in this precision
// (rank <= 1, or det M < 0 with nearly equal smaller singular values).
template <typename T>
__device__ __forceinline__ bool polar_so3(const T M[9], T R[9], int sweeps) {
  T S[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S[3 * r + c] = M[r] * M[c] + M[3 + r] * M[3 + c] + M[6 + r] * M[6 + c];
  T V[9];
  jacobi3(S, V, sweeps);
  T lam[3] = {S[0], S[4], S[8]};
  if (lam[0] < lam[1]) swap_col(V, lam, 0, 1);
  if (lam[1] < lam[2]) swap_col(V, lam, 1, 2);
  if (lam[0] < lam[1]) swap_col(V, lam, 0, 1);
  T v1[3] = {V[0], V[3], V[6]}, v2[3] = {V[1], V[4], V[7]}, v3[3];
  cross3(v1, v2, v3);
  T m1[3], m2[3];
  matvec3(M, v1, m1);
  matvec3(M, v2, m2);
  T n1 = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
  T i1 = drsqrt(n1);
  T u1[3] = {m1[0] * i1, m1[1] * i1, m1[2] * i1};
  T d = u1[0] * m2[0] + u1[1] * m2[1] + u1[2] * m2[2];
  T w2[3] = {m2[0] - d * u1[0], m2[1] - d * u1[1], m2[2] - d * u1[2]};
  T n2 = w2[0] * w2[0] + w2[1] * w2[1] + w2[2] * w2[2];
  T i2 = drsqrt(n2);
  T u2[3] = {w2[0] * i2, w2[1] * i2, w2[2] * i2};
  T u3[3];
  cross3(u1, u2, u3);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[3 * r + c] = u1[r] * v1[c] + u2[r] * v2[c] + u3[r] * v3[c];
  polar_newton(M, R);
  T detM = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
  bool ok = (lam[1] > T(1e-6) * lam[0]) && (lam[0] > T(0));
  if (detM < T(0)) ok = ok && (lam[1] - lam[2] > T(2e-3) * lam[0]);
  return ok;
}

// ---------------------------------------------------------------------------
// 6x6 symmetric positive definite solve by Cholesky (packed lower triangle,
// index i*(i+1)/2 + j for i >= j).  Returns false on a non-positive pivot.
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <typename T>
__device__ __forceinline__ bool chol6_factor(const T A[21], T L[21], T dinv[6]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T d = A[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[tri(j, k)] * L[tri(j, k)];
    if (!(d > T(0))) return false;
    T r = drsqrt(d);
    dinv[j] = r;
    L[tri(j, j)] = d * r;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      T v = A[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= L[tri(i, k)] * L[tri(j, k)];
      L[tri(i, j)] = v * r;
    }
  }
  return true;
}

template <typename T>
__device__ __forceinline__ void chol6_subst(const T L[21], const T dinv[6], const T g[6], T x[6]) {
  T y[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T v = g[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= L[tri(i, k)] * y[k];
    y[i] = v * dinv[i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    T v = y[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) v -= L[tri(k, i)] * x[k];
    x[i] = v * dinv[i];
  }
}

template <typename T>
__device__ __forceinline__ bool chol6_solve(const T A[21], const T g[6], T x[6]) {
  T L[21], dinv[6];
  if (!chol6_factor<T>(A, L, dinv)) return false;
  chol6_subst<T>(L, dinv, g, x);
  return true;
}

// The same solve in dual numbers: the values as above; the derivative of
// x = A^{-1} g is A^{-1} (g' - A' x), solved with the same factor.
template <typename T>
__device__ __forceinline__ bool chol6_solve(const Dual<T> A[21], const Dual<T> g[6], Dual<T> x[6]) {
  T Av[21], gv[6], xv[6], L[21], dinv[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) Av[k] = A[k].v;
#pragma unroll
  for (int k = 0; k < 6; ++k) gv[k] = g[k].v;
  if (!chol6_factor<T>(Av, L, dinv)) return false;
  chol6_subst<T>(L, dinv, gv, xv);
  T r[6], xd[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T v = g[i].d;
#pragma unroll
    for (int j = 0; j < 6; ++j) v -= A[i >= j ? tri(i, j) : tri(j, i)].d * xv[j];
    r[i] = v;
  }
  chol6_subst<T>(L, dinv, r, xd);
#pragma unroll
  for (int k = 0; k < 6; ++k) x[k] = Dual<T>(xv[k], xd[k]);
  return true;
}

// ---------------------------------------------------------------------------
// Whitened Gauss-Newton terms of one 2D-3D keypoint.
//   P: camera-frame point, pt = P - pivot, iz = 1/P.z,
//   whitening U = [[w0, w1], [0, w2]] with U^T U = Lambda,
//   rt: whitened residual U (q - u).
// The Jacobian of the pixel u under the left update about the pivot is
// dPi/dP * [-[pt]x | I]; whitened rows are [pt x d_k | d_k] with
// d_0 = (w0 fx iz, w1 fy iz, -(w0 fx X + w1 fy Y) iz^2), d_1 = (0, w2 fy iz, -w2 fy Y iz^2).
template <typename T>
__device__ __forceinline__ void gn_accumulate(const T P[3], const T pt[3], T iz, T fx, T fy,
                                              const T w[3], T rt0, T rt1, T A[21], T g[6]) {
  T a = fx * iz, c = fy * iz;
  T nx = P[0] * iz, ny = P[1] * iz;
  T d0[3] = {w[0] * a, w[1] * c, -(w[0] * a * nx + w[1] * c * ny)};
  T d1[3] = {T(0), w[2] * c, -w[2] * c * ny};
  T j0[6], j1[6];
  cross3(pt, d0, j0);
  j0[3] = d0[0];
  j0[4] = d0[1];
  j0[5] = d0[2];
  j1[0] = pt[1] * d1[2] - pt[2] * d1[1];
  j1[1] = -pt[0] * d1[2];
  j1[2] = pt[0] * d1[1];
  j1[3] = T(0);
  j1[4] = d1[1];
  j1[5] = d1[2];
  // one multiply-add per nonzero product, chained into the accumulator
  // (j1[3] is structurally zero)
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int k = 0; k <= i; ++k) {
      A[tri(i, k)] += j0[i] * j0[k];
      if (i != 3 && k != 3) A[tri(i, k)] += j1[i] * j1[k];
    }
    g[i] += j0[i] * rt0;
    if (i != 3) g[i] += j1[i] * rt1;
  }
}

// Left update about the pivot o: R <- E R, t <- E (t - o) + o + dv, E = Exp(dw).
template <typename T>
__device__ __forceinline__ void apply_update(const T x[6], const T o[3], T R[9], T t[3]) {
  T E[9], Rn[9], d[3], e[3];
  exp_so3(x, E);
  matmul3(E, R, Rn);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = Rn[k];
  d[0] = t[0] - o[0];
  d[1] = t[1] - o[1];
  d[2] = t[2] - o[2];
  matvec3(E, d, e);
  t[0] = e[0] + o[0] + x[3];
  t[1] = e[1] + o[1] + x[4];
  t[2] = e[2] + o[2] + x[5];
}

// ---------------------------------------------------------------------------
// unit quaternions (w, x, y, z)
__device__ __forceinline__ float4 quat_mul(float4 a, float4 b) {
  return make_float4(a.x * b.x - a.y * b.y - a.z * b.z - a.w * b.w,
                     a.x * b.y + a.y * b.x + a.z * b.w - a.w * b.z,
                     a.x * b.z - a.y * b.w + a.z * b.x + a.w * b.y,
                     a.x * b.w + a.y * b.z - a.z * b.y + a.w * b.x);
}

// Rotation matrix -> unit quaternion (Shepperd's largest-component branch),
// stored as float4 (x = w, y = qx, z = qy, w = qz), sign chosen with w >= 0.
__device__ __forceinline__ float4 quat_from_rot(const float R[9]) {
  float tr = R[0] + R[4] + R[8];
  float qw, qx, qy, qz;
  if (tr > 0.f) {
    float s = sqrtf(tr + 1.f) * 2.f;
    qw = 0.25f * s;
    qx = (R[7] - R[5]) / s;
    qy = (R[2] - R[6]) / s;
    qz = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    float s = sqrtf(1.f + R[0] - R[4] - R[8]) * 2.f;
    qw = (R[7] - R[5]) / s;
    qx = 0.25f * s;
    qy = (R[1] + R[3]) / s;
    qz = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    float s = sqrtf(1.f + R[4] - R[0] - R[8]) * 2.f;
    qw = (R[2] - R[6]) / s;
    qx = (R[1] + R[3]) / s;
    qy = 0.25f * s;
    qz = (R[5] + R[7]) / s;
  } else {
    float s = sqrtf(1.f + R[8] - R[0] - R[4]) * 2.f;
    qw = (R[3] - R[1]) / s;
    qx = (R[2] + R[6]) / s;
    qy = (R[5] + R[7]) / s;
    qz = 0.25f * s;
  }
  float n = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  if (qw < 0.f) n = -n;
  return make_float4(qw * n, qx * n, qy * n, qz * n);
}

__device__ __forceinline__ void rot_from_quat(float4 q, float R[9]) {
  float w = q.x, x = q.y, y = q.z, z = q.w;
  R[0] = 1.f - 2.f * (y * y + z * z);
  R[1] = 2.f * (x * y - w * z);
  R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z);
  R[4] = 1.f - 2.f * (x * x + z * z);
  R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y);
  R[7] = 2.f * (y * z + w * x);
  R[8] = 1.f - 2.f * (x * x + y * y);
}

}  // namespace purse
