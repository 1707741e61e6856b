// Step I of the paper ("The CLOSURE Algorithm"): candidate start poses, each
// kept when it lies in S.  One trial per lane; instance j runs M_j trials
// (its sample count in the batch).
//
// - 3D-3D (random sample averaging with a minimal solver): three distinct
//   correspondences, a random point inside each of their balls, Arun's
//   method on the three pairs.
// - 2D-3D: three distinct correspondences, a random point inside each of
//   their ellipses, and the perspective-3-point problem for the three
//   bearing rays: with s2 = u s1 and s3 = v s1 along the rays, the law of
//   cosines for the three pairs gives u = N(v) / D(v) and a quartic in v;
//   its real roots (found by bracketing between the roots of its
//   derivatives and bisection, in float64) give the camera points, and Arun's
//   method the pose.  Roots are taken in increasing v; the first solution
//   in S is kept.
// - pose regression (eq. PURSEregression): a random convex combination of
//   the hypotheses, R = proj_SO3(sum w_i R_i), t = sum w_i t_i, with weights
//   uniform on the simplex.
//
// Random numbers: Philox4x64-10; pose regression key (seed, 3), counter
// (trial, i, 0, 0), word 0 for the weight of hypothesis i; the keypoint
// sets key (seed, 4), counter (trial, k, 0, 0): k = 0 picks the
// correspondences, k = 1..3 the point in the k-th constraint.
#include "purse_fit.hpp"
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

namespace {

constexpr int kInitBlock = 256;

__device__ __forceinline__ void philox_u3(uint64_t seed, uint64_t key1, uint64_t c0, uint64_t c1, double u[3]) {
  uint64_t c[4] = {c0, c1, 0ull, 0ull};
  philox4x64_10(c, seed, key1);
  for (int q = 0; q < 3; ++q) u[q] = (double)(c[q] >> 40) * 0x1p-24;
}

// True unless the three points are collinear (to float64 resolution).
__device__ __forceinline__ bool has_area(const double P[3][3]) {
  double e1[3], e2[3];
  for (int r = 0; r < 3; ++r) {
    e1[r] = P[1][r] - P[0][r];
    e2[r] = P[2][r] - P[0][r];
  }
  const double c0 = e1[1] * e2[2] - e1[2] * e2[1], c1 = e1[2] * e2[0] - e1[0] * e2[2],
               c2 = e1[0] * e2[1] - e1[1] * e2[0];
  const double n1 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
  const double n2 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
  return c0 * c0 + c1 * c1 + c2 * c2 > 1e-24 * n1 * n2;
}

// Arun's method on three pairs P_k -> X_k (float64): R = proj_SO3(sum
// (X_k - Xbar)(P_k - Pbar)^T), t = Xbar - R Pbar.  False if degenerate.
__device__ bool arun3(const double P[3][3], const double X[3][3], double R[9], double t[3]) {
  double pb[3] = {0, 0, 0}, xb[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k)
    for (int r = 0; r < 3; ++r) {
      pb[r] += P[k][r] / 3.0;
      xb[r] += X[k][r] / 3.0;
    }
  double H[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 3; ++k)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) H[3 * r + c] += (X[k][r] - xb[r]) * (P[k][c] - pb[c]);
  // Three pairs give a rank-two H whose determinant is zero up to rounding,
  // so polar_so3's flag for "det < 0 with close smaller singular values"
  // says nothing here: the polar factor u1 v1^T + u2 v2^T + (u1 x u2)(v1 x
  // v2)^T is well defined whenever both triangles have area.
  polar_so3<double>(H, R, 12);
  for (int r = 0; r < 3; ++r) t[r] = xb[r] - (R[3 * r] * pb[0] + R[3 * r + 1] * pb[1] + R[3 * r + 2] * pb[2]);
  // collinear points (a rank-one H) leave the rotation about their line open
  return has_area(P) && has_area(X);
}

// Three distinct indices of n, in the order drawn.
__device__ __forceinline__ void pick_three(const double u[3], int n, int idx[3]) {
  int taken[3];
  for (int q = 0; q < 3; ++q) {
    int x = (int)floor(u[q] * (double)(n - q));
    // skip the indices already taken, smallest first
    int s0 = q > 0 ? taken[0] : INT32_MAX, s1 = q > 1 ? taken[1] : INT32_MAX;
    if (s1 < s0) {
      const int tmp = s0;
      s0 = s1;
      s1 = tmp;
    }
    if (x >= s0) ++x;
    if (x >= s1) ++x;
    taken[q] = x;
    idx[q] = x;
  }
}

__device__ __forceinline__ double polyval(const double *c, int deg, double x) {
  double v = c[0];
  for (int k = 1; k <= deg; ++k) v = v * x + c[k];
  return v;
}

// Real roots of a polynomial of degree <= 4 (highest coefficient first),
// ascending: the roots of its derivative bracket the monotone pieces, each
// bisected to float64 resolution (every degree handled the same way).
__device__ int real_roots4(const double *c4, double roots[4]) {
  double c[5][5];  // c[d]: the (4 - d)-th derivative's coefficients, degree d
  for (int k = 0; k <= 4; ++k) c[4][k] = c4[k];
  for (int d = 4; d > 1; --d)
    for (int k = 0; k < d; ++k) c[d - 1][k] = c[d][k] * (double)(d - k);
  // bound on every root (Cauchy) of the quartic
  double lead = c[4][0];
  if (lead == 0.0) return 0;
  double B = 0.0;
  for (int k = 1; k <= 4; ++k) B = fmax(B, fabs(c[4][k] / lead));
  B += 1.0;
  double r[4];
  int nr = 0;
  // degree 1
  if (c[1][0] != 0.0) {
    r[0] = -c[1][1] / c[1][0];
    nr = 1;
  }
  for (int d = 2; d <= 4; ++d) {
    double pts[6];
    int np = 0;
    pts[np++] = -B;
    for (int k = 0; k < nr; ++k)
      if (r[k] > -B && r[k] < B) pts[np++] = r[k];
    pts[np++] = B;
    int nn = 0;
    double rn[4];
    for (int k = 0; k + 1 < np; ++k) {
      double lo = pts[k], hi = pts[k + 1];
      double flo = polyval(c[d], d, lo), fhi = polyval(c[d], d, hi);
      if (flo == 0.0) {
        if (nn == 0 || rn[nn - 1] != lo) rn[nn++] = lo;
        continue;
      }
      if ((flo < 0.0) == (fhi < 0.0)) continue;
      for (int it = 0; it < 100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double fm = polyval(c[d], d, mid);
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      if (nn < 4) rn[nn++] = 0.5 * (lo + hi);
    }
    nr = nn;
    for (int k = 0; k < nn; ++k) r[k] = rn[k];
  }
  for (int k = 0; k < nr; ++k) roots[k] = r[k];
  return nr;
}

// Polynomial helpers (highest degree first, fixed storage of 5).
__device__ __forceinline__ void pmul(const double *a, int da, const double *b, int db, double *out) {
  for (int k = 0; k <= da + db; ++k) out[k] = 0.0;
  for (int i = 0; i <= da; ++i)
    for (int jj = 0; jj <= db; ++jj) out[i + jj] += a[i] * b[jj];
}

// R_i of a pose-regression hypothesis from its stored quaternion (w, x, y,
// z), normalised, in float64.
__device__ void hyp_rotation(const float *q4, double R[9]) {
  const double q0 = q4[0], q1 = q4[1], q2 = q4[2], q3 = q4[3];
  const double s = 1.0 / sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
  const double w = q0 * s, x = q1 * s, y = q2 * s, z = q3 * s;
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

struct InitKp {
  const float *a, *c, *L, *beta;
};

// in_purse of (R, t) against every constraint of the instance (float64, the
// sampler's test with tolerance tau and depth > z_min).
__device__ bool in_s_keypoints(int kind, int n, const InitKp &kp, const float K[4], const double R[9],
                               const double t[3], double tau, double z_min) {
  for (int i = 0; i < n; ++i) {
    double P[3];
    for (int r = 0; r < 3; ++r)
      P[r] = R[3 * r] * kp.a[3 * i] + R[3 * r + 1] * kp.a[3 * i + 1] + R[3 * r + 2] * kp.a[3 * i + 2] + t[r];
    double rr;
    if (kind == PURSE_KIND_2D3D) {
      if (!(P[2] > z_min)) return false;
      const double e0 = K[0] * P[0] / P[2] + K[2] - kp.c[3 * i];
      const double e1 = K[1] * P[1] / P[2] + K[3] - kp.c[3 * i + 1];
      const float *l = kp.L + 4 * i;
      rr = sqrt(fmax(0.0, e0 * (l[0] * e0 + l[1] * e1) + e1 * (l[2] * e0 + l[3] * e1)));
    } else {
      const double e0 = P[0] - kp.c[3 * i], e1 = P[1] - kp.c[3 * i + 1], e2 = P[2] - kp.c[3 * i + 2];
      rr = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    }
    if (!(rr <= (double)kp.beta[i] + tau)) return false;
  }
  return true;
}

}  // namespace

__global__ void __launch_bounds__(kInitBlock) k_init(DevBatch b, DevParams p, float *poses, uint8_t *mask) {
  const int j = blockIdx.y;
  int64_t off, M;
  sample_range(b.sample_off, j, b.total_samples, b.max_samples, off, M);
  const int64_t s = (int64_t)blockIdx.x * kInitBlock + threadIdx.x;
  if (s >= M) return;
  const int kind = b.kind[j];
  const int n = b.n_kp[j];
  const int64_t ko = b.kp_off[j];
  const uint64_t seed = b.seed[j];
  float *out = poses + 12 * (off + s);
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, t[3] = {0, 0, 0};
  bool ok = false;
  const bool valid = n >= (kind == PURSE_KIND_REG ? 1 : 3) && n <= PURSE_MAX_KP && ko >= 0 &&
                     b.kp_off[j + 1] - ko == n && b.kp_off[j + 1] <= b.total_kp;
  const InitKp kp{b.model_pts + 3 * ko, b.centres + 3 * ko, b.shapes + 4 * ko, b.bounds + ko};
  if (valid && kind == PURSE_KIND_REG) {
    // convex combination of the hypotheses
    double M9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, wsum = 0.0;
    double tt[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
      double u[3];
      philox_u3(seed, 3ull, (uint64_t)s, (uint64_t)i, u);
      const double w = -log1p(-u[0]);
      double Ri[9];
      hyp_rotation(kp.L + 4 * i, Ri);
      for (int k = 0; k < 9; ++k) M9[k] += w * Ri[k];
      for (int r = 0; r < 3; ++r) tt[r] += w * kp.c[3 * i + r];
      wsum += w;
    }
    for (int k = 0; k < 9; ++k) M9[k] /= wsum;
    for (int r = 0; r < 3; ++r) t[r] = tt[r] / wsum;
    polar_so3<double>(M9, R, 12);
    ok = true;
    const double tau = p.tau3;
    for (int i = 0; i < n && ok; ++i) {
      double Ri[9];
      hyp_rotation(kp.L + 4 * i, Ri);
      double f = 0.0;
      for (int k = 0; k < 9; ++k) f += (R[k] - Ri[k]) * (R[k] - Ri[k]);
      double e2 = 0.0;
      for (int r = 0; r < 3; ++r) e2 += (t[r] - kp.c[3 * i + r]) * (t[r] - kp.c[3 * i + r]);
      ok = sqrt(f) <= (double)kp.a[3 * i] + tau && sqrt(e2) <= (double)kp.beta[i] + tau;
    }
  } else if (valid && (kind == PURSE_KIND_3D3D || kind == PURSE_KIND_2D3D)) {
    double u[3];
    philox_u3(seed, 4ull, (uint64_t)s, 0ull, u);
    int idx[3];
    pick_three(u, n, idx);
    double Pm[3][3];
    for (int k = 0; k < 3; ++k)
      for (int r = 0; r < 3; ++r) Pm[k][r] = kp.a[3 * idx[k] + r];
    const bool is2d = kind == PURSE_KIND_2D3D;
    float K[4] = {0, 0, 0, 0};
    if (is2d)
      for (int q = 0; q < 4; ++q) K[q] = b.intrinsics[4 * j + q];
    const double tau = is2d ? p.tau2 : p.tau3;
    if (!is2d) {
      double X[3][3];
      for (int k = 0; k < 3; ++k) {
        philox_u3(seed, 4ull, (uint64_t)s, (uint64_t)(k + 1), u);
        const double z = 1.0 - 2.0 * u[0];
        const double rho = sqrt(fmax(0.0, 1.0 - z * z));
        double sp, cp;
        sincospi(2.0 * u[1], &sp, &cp);
        const double rad = cbrt(u[2]) * (double)kp.beta[idx[k]];
        const double d[3] = {rho * cp, rho * sp, z};
        for (int r = 0; r < 3; ++r) X[k][r] = (double)kp.c[3 * idx[k] + r] + rad * d[r];
      }
      ok = arun3(Pm, X, R, t) && in_s_keypoints(kind, n, kp, K, R, t, tau, (double)p.z_min);
    } else {
      // a point inside each ellipse, its bearing
      double f[3][3];
      for (int k = 0; k < 3; ++k) {
        philox_u3(seed, 4ull, (uint64_t)s, (uint64_t)(k + 1), u);
        double sp, cp;
        sincospi(2.0 * u[1], &sp, &cp);
        const double rad = sqrt(u[2]) * (double)kp.beta[idx[k]];
        const float *l = kp.L + 4 * idx[k];
        // U^T U = Lambda, U = [[w0, w1], [0, w2]]; e = U^-1 y
        const double w0 = sqrt((double)l[0]), w1 = (double)l[1] / w0;
        const double w2 = sqrt(fmax(0.0, (double)l[3] - w1 * w1));
        const double y0 = rad * cp, y1 = rad * sp;
        const double e1 = y1 / w2, e0 = (y0 - w1 * e1) / w0;
        const double px = (double)kp.c[3 * idx[k]] + e0, py = (double)kp.c[3 * idx[k] + 1] + e1;
        double d[3] = {(px - K[2]) / K[0], (py - K[3]) / K[1], 1.0};
        const double nd = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int r = 0; r < 3; ++r) f[k][r] = d[r] * nd;
      }
      double dd[3];
      for (int r = 0; r < 3; ++r) dd[r] = Pm[1][r] - Pm[2][r];
      const double a = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      for (int r = 0; r < 3; ++r) dd[r] = Pm[0][r] - Pm[2][r];
      const double bb = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      for (int r = 0; r < 3; ++r) dd[r] = Pm[0][r] - Pm[1][r];
      const double c = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      const double ca = f[1][0] * f[2][0] + f[1][1] * f[2][1] + f[1][2] * f[2][2];
      const double cb = f[0][0] * f[2][0] + f[0][1] * f[2][1] + f[0][2] * f[2][2];
      const double cg = f[0][0] * f[1][0] + f[0][1] * f[1][1] + f[0][2] * f[1][2];
      const double Kc = (a * a - c * c) / (bb * bb);
      // q = v^2 - 2 cb v + 1; N = K q + 1 - v^2; D = -2 ca v + 2 cg
      const double q[3] = {1.0, -2.0 * cb, 1.0};
      const double N[3] = {Kc - 1.0, -2.0 * cb * Kc, Kc + 1.0};
      const double D[2] = {-2.0 * ca, 2.0 * cg};
      double DD[3], NN[5], ND[4], qDD[5];
      pmul(D, 1, D, 1, DD);
      pmul(N, 2, N, 2, NN);
      pmul(N, 2, D, 1, ND);
      pmul(q, 2, DD, 2, qDD);
      const double k2 = (c * c) / (bb * bb);
      double quart[5];
      for (int k = 0; k <= 4; ++k) {
        double v = NN[k] - k2 * qDD[k];
        if (k >= 1) v += -2.0 * cg * ND[k - 1];
        if (k >= 2) v += DD[k - 2];
        quart[k] = v;
      }
      double roots[4];
      const int nr = real_roots4(quart, roots);
      for (int k = 0; k < nr && !ok; ++k) {
        const double v = roots[k];
        if (!(v > 0.0)) continue;
        const double Dv = D[0] * v + D[1];
        if (fabs(Dv) < 1e-14) continue;
        const double uu = polyval(N, 2, v) / Dv;
        const double qv = polyval(q, 2, v);
        if (!(uu > 0.0) || !(qv > 0.0)) continue;
        const double s1 = bb / sqrt(qv);
        double X[3][3];
        for (int r = 0; r < 3; ++r) {
          X[0][r] = s1 * f[0][r];
          X[1][r] = uu * s1 * f[1][r];
          X[2][r] = v * s1 * f[2][r];
        }
        double Rk[9], tk[3];
        if (!arun3(Pm, X, Rk, tk)) continue;
        if (in_s_keypoints(kind, n, kp, K, Rk, tk, tau, (double)p.z_min)) {
          for (int q2 = 0; q2 < 9; ++q2) R[q2] = Rk[q2];
          for (int r = 0; r < 3; ++r) t[r] = tk[r];
          ok = true;
        }
      }
    }
  }
  float4 *o4 = reinterpret_cast<float4 *>(out);
  o4[0] = make_float4((float)R[0], (float)R[1], (float)R[2], (float)R[3]);
  o4[1] = make_float4((float)R[4], (float)R[5], (float)R[6], (float)R[7]);
  o4[2] = make_float4((float)R[8], (float)t[0], (float)t[1], (float)t[2]);
  mask[off + s] = ok ? PURSE_MASK_FEASIBLE : 0;
}

void launch_init(const DevBatch &b, const DevParams &p, float *poses, uint8_t *mask, hipStream_t stream) {
  const dim3 grid((unsigned)((b.max_samples + kInitBlock - 1) / kInitBlock), (unsigned)b.n_inst);
  hipLaunchKernelGGL(k_init, grid, dim3(kInitBlock), 0, stream, b, p, poses, mask);
}

}  // namespace purse
