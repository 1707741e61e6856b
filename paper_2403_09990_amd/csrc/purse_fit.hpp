// Centre-fit building blocks shared by the prologue and the backward: DLT
// and weak-perspective starts, whitening of Lambda, the Gauss-Newton fit of
// the 2D-3D maximum-likelihood pose, Arun's fit for 3D-3D.
#pragma once

#include "purse_device.hpp"

namespace purse {

__device__ inline bool finite_f(float x) { return isfinite(x); }



// 12x12 symmetric positive definite helpers for the DLT (packed lower).
__device__ __forceinline__ int tri12(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ inline bool chol12(double *L /* 78, in: A, out: L */) {
  for (int j = 0; j < 12; ++j) {
    double d = L[tri12(j, j)];
    for (int k = 0; k < j; ++k) d -= L[tri12(j, k)] * L[tri12(j, k)];
    if (!(d > 0.0)) return false;
    double r = sqrt(d);
    L[tri12(j, j)] = r;
    for (int i = j + 1; i < 12; ++i) {
      double v = L[tri12(i, j)];
      for (int k = 0; k < j; ++k) v -= L[tri12(i, k)] * L[tri12(j, k)];
      L[tri12(i, j)] = v / r;
    }
  }
  return true;
}

__device__ inline void chol12_solve(const double *L, double *x /* in: rhs, out: solution */) {
  for (int i = 0; i < 12; ++i) {
    double v = x[i];
    for (int k = 0; k < i; ++k) v -= L[tri12(i, k)] * x[k];
    x[i] = v / L[tri12(i, i)];
  }
  for (int i = 11; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < 12; ++k) v -= L[tri12(k, i)] * x[k];
    x[i] = v / L[tri12(i, i)];
  }
}

// Direct linear transform in normalised image coordinates, model points
// centred and scaled for conditioning; the null vector of the 2N x 12 system
// comes from inverse iteration on its normal matrix.  Returns (R, t) with the
// sign fixed by det(P[:, :3]) > 0 and t = P[:, 3] / (mean singular value).
__device__ inline bool dlt_2d(const float *Z, const float *z, int n, const float K[4], double R[9], double t[3]) {
  double zb[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) zb[r] += Z[3 * i + r];
  for (int r = 0; r < 3; ++r) zb[r] /= n;
  double ss = 0;
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) ss += (Z[3 * i + r] - zb[r]) * (Z[3 * i + r] - zb[r]);
  double sc = sqrt(ss / n);
  if (!(sc > 0)) return false;
  double L[78];
  for (int k = 0; k < 78; ++k) L[k] = 0;
  for (int i = 0; i < n; ++i) {
    double xn = ((double)z[3 * i] - K[2]) / K[0];
    double yn = ((double)z[3 * i + 1] - K[3]) / K[1];
    double h[4] = {(Z[3 * i] - zb[0]) / sc, (Z[3 * i + 1] - zb[1]) / sc, (Z[3 * i + 2] - zb[2]) / sc, 1.0};
    double r1[12], r2[12];
    for (int c = 0; c < 4; ++c) {
      r1[c] = -h[c];
      r1[4 + c] = 0;
      r1[8 + c] = xn * h[c];
      r2[c] = 0;
      r2[4 + c] = -h[c];
      r2[8 + c] = yn * h[c];
    }
    for (int a = 0; a < 12; ++a)
      for (int b = 0; b <= a; ++b) L[tri12(a, b)] += r1[a] * r1[b] + r2[a] * r2[b];
  }
  double tr = 0;
  for (int a = 0; a < 12; ++a) tr += L[tri12(a, a)];
  for (int a = 0; a < 12; ++a) L[tri12(a, a)] += 1e-13 * tr;
  if (!chol12(L)) return false;
  double v[12];
  for (int a = 0; a < 12; ++a) v[a] = 1.0 + 0.01 * a;
  // until the unit iterate moves by less than 1e-14 (a start for the
  // Gauss-Newton fit, which converges from it), at most 80 solves
  for (int it = 0; it < 80; ++it) {
    double u[12];
    for (int a = 0; a < 12; ++a) u[a] = v[a];
    chol12_solve(L, v);
    double nn = 0;
    for (int a = 0; a < 12; ++a) nn += v[a] * v[a];
    nn = 1.0 / sqrt(nn);
    double dv = 0;
    for (int a = 0; a < 12; ++a) {
      v[a] *= nn;
      dv = fmax(dv, fabs(v[a] - u[a]));
    }
    if (it >= 2 && dv <= 1e-14) break;
  }
  // undo the model normalisation: P = P' [[I/sc, -zb/sc], [0, 1]]
  double P[12];
  for (int r = 0; r < 3; ++r) {
    double acc = v[4 * r + 3];
    for (int c = 0; c < 3; ++c) {
      P[4 * r + c] = v[4 * r + c] / sc;
      acc -= v[4 * r + c] * zb[c] / sc;
    }
    P[4 * r + 3] = acc;
  }
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[3 * r + c] = P[4 * r + c];
  double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
               M[2] * (M[3] * M[7] - M[4] * M[6]);
  if (det < 0) {
    for (int k = 0; k < 12; ++k) P[k] = -P[k];
    for (int k = 0; k < 9; ++k) M[k] = -M[k];
  }
  double S[9], V[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) S[3 * r + c] = M[r] * M[c] + M[3 + r] * M[3 + c] + M[6 + r] * M[6 + c];
  jacobi3<double>(S, V, 12);
  double s = (sqrt(fmax(S[0], 0.0)) + sqrt(fmax(S[4], 0.0)) + sqrt(fmax(S[8], 0.0))) / 3.0;
  if (!(s > 0)) return false;
  polar_so3<double>(M, R, 12);
  for (int r = 0; r < 3; ++r) t[r] = P[4 * r + 3] / s;
  return true;
}

// Weak-perspective initialisation: least squares x_n = A Z + b (a scaled
// orthographic camera) by the 4x4 normal equations; s = mean row norm of A,
// R = proj_SO3 [A0/s; A1/s; A0 x A1 / s^2], t = (b / s, 1 / s).
__device__ inline bool affine_2d(const float *Z, const float *z, int n, const float K[4], double R[9], double t[3]) {
  double G[16], r0[4], r1[4];
  for (int k = 0; k < 16; ++k) G[k] = 0;
  for (int k = 0; k < 4; ++k) r0[k] = r1[k] = 0;
  for (int i = 0; i < n; ++i) {
    double x[4] = {Z[3 * i], Z[3 * i + 1], Z[3 * i + 2], 1.0};
    double xn = ((double)z[3 * i] - K[2]) / K[0];
    double yn = ((double)z[3 * i + 1] - K[3]) / K[1];
    for (int a = 0; a < 4; ++a) {
      for (int b = 0; b < 4; ++b) G[4 * a + b] += x[a] * x[b];
      r0[a] += x[a] * xn;
      r1[a] += x[a] * yn;
    }
  }
  // Cholesky of G (4x4) and two solves
  double L[16];
  for (int k = 0; k < 16; ++k) L[k] = 0;
  for (int j = 0; j < 4; ++j) {
    double d = G[4 * j + j];
    for (int k = 0; k < j; ++k) d -= L[4 * j + k] * L[4 * j + k];
    if (!(d > 0)) return false;
    L[4 * j + j] = sqrt(d);
    for (int i = j + 1; i < 4; ++i) {
      double v = G[4 * i + j];
      for (int k = 0; k < j; ++k) v -= L[4 * i + k] * L[4 * j + k];
      L[4 * i + j] = v / L[4 * j + j];
    }
  }
  double *rhs[2] = {r0, r1};
  for (int c = 0; c < 2; ++c) {
    double *x = rhs[c];
    for (int i = 0; i < 4; ++i) {
      double v = x[i];
      for (int k = 0; k < i; ++k) v -= L[4 * i + k] * x[k];
      x[i] = v / L[4 * i + i];
    }
    for (int i = 3; i >= 0; --i) {
      double v = x[i];
      for (int k = i + 1; k < 4; ++k) v -= L[4 * k + i] * x[k];
      x[i] = v / L[4 * i + i];
    }
  }
  double a0[3] = {r0[0], r0[1], r0[2]}, a1[3] = {r1[0], r1[1], r1[2]};
  double s = 0.5 * (sqrt(a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2]) +
                    sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]));
  if (!(s > 0)) return false;
  double c3[3];
  cross3(a0, a1, c3);
  double M[9] = {a0[0] / s, a0[1] / s, a0[2] / s, a1[0] / s, a1[1] / s, a1[2] / s,
                 c3[0] / (s * s), c3[1] / (s * s), c3[2] / (s * s)};
  polar_so3<double>(M, R, 12);
  t[0] = r0[3] / s;
  t[1] = r1[3] / s;
  t[2] = 1.0 / s;
  return true;
}

// Whitening factor U = [[u00, u01], [0, u11]] with U^T U = Lambda.
template <typename T>
__device__ __forceinline__ void whiten_factor(const float *Lam, T w[3]) {
  T l00 = Lam[0], l01 = Lam[1], l11 = Lam[3];
  w[0] = sqrt((double)l00);
  w[1] = l01 / w[0];
  w[2] = sqrt((double)(l11 - w[1] * w[1]));
}

// Gauss-Newton centre fit of the 2D-3D maximum-likelihood pose (eq. MLE with
// rho = ||.||^2_Lambda): targets are the ellipse centres, each step about the
// pivot R Zbar + t of the current pose, iterated until the step is below
// kCentreTol (rotation) and kCentreTol (1 + |t|_inf) (translation), at most
// `steps` times.  T is double, or a dual number when the backward
// differentiates the fit; obs(i, z, w) gives keypoint i's image point and
// whitening factor.
constexpr double kCentreTol = 1e-13;

template <typename T, typename OBS>
__device__ bool gn_centre_2d(const float *Z, const OBS &obs, int n, const float K[4], int steps, double z_min,
                             T R[9], T t[3]) {
  double zb[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) zb[r] += Z[3 * i + r];
  for (int r = 0; r < 3; ++r) zb[r] /= n;
  const double Kd[4] = {K[0], K[1], K[2], K[3]};
  for (int st = 0; st < steps; ++st) {
    T o[3];
    for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * zb[0] + R[3 * r + 1] * zb[1] + R[3 * r + 2] * zb[2] + t[r];
    T A[21], g[6];
    for (int k = 0; k < 21; ++k) A[k] = T(0.0);
    for (int k = 0; k < 6; ++k) g[k] = T(0.0);
    for (int i = 0; i < n; ++i) {
      T P[3];
      for (int r = 0; r < 3; ++r)
        P[r] = R[3 * r] * (double)Z[3 * i] + R[3 * r + 1] * (double)Z[3 * i + 1] + R[3 * r + 2] * (double)Z[3 * i + 2] + t[r];
      if (!(value_of(P[2]) > z_min)) return false;
      T iz = T(1.0) / P[2];
      T u = Kd[0] * (P[0] * iz) + Kd[2], v = Kd[1] * (P[1] * iz) + Kd[3];
      T z[2], w[3];
      obs(i, z, w);
      T r0 = z[0] - u, r1 = z[1] - v;
      T rt0 = w[0] * r0 + w[1] * r1, rt1 = w[2] * r1;
      T pt[3] = {P[0] - o[0], P[1] - o[1], P[2] - o[2]};
      gn_accumulate<T>(P, pt, iz, T(Kd[0]), T(Kd[1]), w, rt0, rt1, A, g);
    }
    T d[6];
    if (!chol6_solve<T>(A, g, d)) return false;
    apply_update<T>(d, o, R, t);
    // converged: the step is at the float64 rounding level of the pose
    double dw = 0.0, dv = 0.0, tm = 0.0;
    for (int k = 0; k < 3; ++k) {
      dw = fmax(dw, fabs(value_of(d[k])));
      dv = fmax(dv, fabs(value_of(d[3 + k])));
      tm = fmax(tm, fabs(value_of(t[k])));
    }
    if (dw <= kCentreTol && dv <= kCentreTol * (1.0 + tm)) break;
  }
  for (int i = 0; i < n; ++i) {
    double pz = value_of(R[6]) * Z[3 * i] + value_of(R[7]) * Z[3 * i + 1] + value_of(R[8]) * Z[3 * i + 2] + value_of(t[2]);
    if (!(pz > z_min)) return false;
  }
  return true;
}

// gn_centre_2d<double> on a whole wavefront, for up to 64 keypoints: lane i
// takes keypoint i, the normal equations are summed over the wavefront by an
// xor butterfly (a fixed order, every lane ends with the same sums) and every
// lane then takes the same step, so the control flow stays wave-uniform.
template <typename OBS>
__device__ bool gn_centre_2d_wave(const float *Z, const OBS &obs, int n, const float K[4], int steps, double z_min,
                                  double R[9], double t[3]) {
  const int lane = threadIdx.x & 63;
  double zb[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) zb[r] += Z[3 * i + r];
  for (int r = 0; r < 3; ++r) zb[r] /= n;
  const double Kd[4] = {K[0], K[1], K[2], K[3]};
  const bool mine = lane < n;
  const int i = mine ? lane : 0;
  const double Zi[3] = {Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]};
  double zi[2], wi[3];
  obs(i, zi, wi);
  for (int st = 0; st < steps; ++st) {
    double o[3];
    for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * zb[0] + R[3 * r + 1] * zb[1] + R[3 * r + 2] * zb[2] + t[r];
    double A[21], g[6];
    for (int k = 0; k < 21; ++k) A[k] = 0.0;
    for (int k = 0; k < 6; ++k) g[k] = 0.0;
    double P[3];
    for (int r = 0; r < 3; ++r) P[r] = R[3 * r] * Zi[0] + R[3 * r + 1] * Zi[1] + R[3 * r + 2] * Zi[2] + t[r];
    if (__ballot(mine && !(P[2] > z_min)) != 0ull) return false;
    if (mine) {
      const double iz = 1.0 / P[2];
      const double u = Kd[0] * (P[0] * iz) + Kd[2], v = Kd[1] * (P[1] * iz) + Kd[3];
      const double r0 = zi[0] - u, r1 = zi[1] - v;
      const double rt0 = wi[0] * r0 + wi[1] * r1, rt1 = wi[2] * r1;
      const double pt[3] = {P[0] - o[0], P[1] - o[1], P[2] - o[2]};
      gn_accumulate<double>(P, pt, iz, Kd[0], Kd[1], wi, rt0, rt1, A, g);
    }
    for (int m = 1; m < 64; m <<= 1) {
      for (int k = 0; k < 21; ++k) A[k] += __shfl_xor(A[k], m, 64);
      for (int k = 0; k < 6; ++k) g[k] += __shfl_xor(g[k], m, 64);
    }
    double d[6];
    if (!chol6_solve<double>(A, g, d)) return false;
    apply_update<double>(d, o, R, t);
    double dw = 0.0, dv = 0.0, tm = 0.0;
    for (int k = 0; k < 3; ++k) {
      dw = fmax(dw, fabs(d[k]));
      dv = fmax(dv, fabs(d[3 + k]));
      tm = fmax(tm, fabs(t[k]));
    }
    if (dw <= kCentreTol && dv <= kCentreTol * (1.0 + tm)) break;
  }
  const double pz = R[6] * Zi[0] + R[7] * Zi[1] + R[8] * Zi[2] + t[2];
  return __ballot(mine && !(pz > z_min)) == 0ull;
}

// Observations of the plain fit: float inputs, whitening from Lambda in float64.
struct ObsPlain {
  const float *z;
  const float *shapes;
  __device__ void operator()(int i, double zz[2], double w[3]) const {
    zz[0] = z[3 * i];
    zz[1] = z[3 * i + 1];
    whiten_factor<double>(shapes + 4 * i, w);
  }
};

// Observations with the whitening factors computed once (3 doubles per
// keypoint, e.g. in LDS): the same values ObsPlain computes on every call.
struct ObsCached {
  const float *z;
  const double *w;
  __device__ void operator()(int i, double zz[2], double ww[3]) const {
    zz[0] = z[3 * i];
    zz[1] = z[3 * i + 1];
    ww[0] = w[3 * i];
    ww[1] = w[3 * i + 1];
    ww[2] = w[3 * i + 2];
  }
};

// Weighted cost sum ||z_i - Pi(R Z_i + t)||^2_Lambda_i of a 2D-3D pose.
template <typename OBS>
__device__ inline double cost_2d_obs(const float *Z, const OBS &obs, int n, const float K[4], const double R[9],
                                     const double t[3]) {
  double c = 0;
  for (int i = 0; i < n; ++i) {
    double m[3] = {Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]}, P[3];
    matvec3(R, m, P);
    for (int r = 0; r < 3; ++r) P[r] += t[r];
    double iz = 1.0 / P[2];
    double u = (double)K[0] * (P[0] * iz) + K[2], v = (double)K[1] * (P[1] * iz) + K[3];
    double zz[2], w[3];
    obs(i, zz, w);
    double r0 = zz[0] - u, r1 = zz[1] - v;
    double a = w[0] * r0 + w[1] * r1, b = w[2] * r1;
    c += a * a + b * b;
  }
  return c;
}

__device__ inline double cost_2d(const float *Z, const float *z, const float *shapes, int n, const float K[4],
                                 const double R[9], const double t[3]) {
  return cost_2d_obs(Z, ObsPlain{z, shapes}, n, K, R, t);
}

// Arun's method in float64: R = proj_SO3(sum (b_i - bbar)(a_i - abar)^T).
__device__ inline void kabsch_centre(const float *a, const float *b, int n, double R[9], double t[3]) {
  double ab[3] = {0, 0, 0}, bb[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) {
      ab[r] += a[3 * i + r];
      bb[r] += b[3 * i + r];
    }
  for (int r = 0; r < 3; ++r) {
    ab[r] /= n;
    bb[r] /= n;
  }
  double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) H[3 * r + c] += ((double)b[3 * i + r] - bb[r]) * ((double)a[3 * i + c] - ab[c]);
  polar_so3<double>(H, R, 12);
  double ra[3];
  matvec3(R, ab, ra);
  for (int r = 0; r < 3; ++r) t[r] = bb[r] - ra[r];
}


}  // namespace purse
