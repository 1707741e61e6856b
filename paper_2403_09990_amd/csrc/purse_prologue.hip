// Per-instance prologue: validation, keypoint records, centre fit (float64),
// pivot and feasible anchor.  One wavefront per instance; the fit is serial
// in lane 0 (it is a few thousand float64 operations per instance).
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

namespace {

__device__ bool finite_f(float x) { return isfinite(x); }

// 12x12 symmetric positive definite helpers for the DLT (packed lower).
__device__ __forceinline__ int tri12(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ bool chol12(double *L /* 78, in: A, out: L */) {
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

__device__ void chol12_solve(const double *L, double *x /* in: rhs, out: solution */) {
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
__device__ bool dlt_2d(const float *Z, const float *z, int n, const float K[4], double R[9], double t[3]) {
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
  for (int it = 0; it < 80; ++it) {
    chol12_solve(L, v);
    double nn = 0;
    for (int a = 0; a < 12; ++a) nn += v[a] * v[a];
    nn = 1.0 / sqrt(nn);
    for (int a = 0; a < 12; ++a) v[a] *= nn;
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
__device__ bool affine_2d(const float *Z, const float *z, int n, const float K[4], double R[9], double t[3]) {
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
// pivot R Zbar + t of the current pose, float64.
__device__ bool gn_centre_2d(const float *Z, const float *z, const float *shapes, int n, const float K[4],
                             int steps, double z_min, double R[9], double t[3]) {
  double zb[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) zb[r] += Z[3 * i + r];
  for (int r = 0; r < 3; ++r) zb[r] /= n;
  const double Kd[4] = {K[0], K[1], K[2], K[3]};
  for (int st = 0; st < steps; ++st) {
    double o[3];
    matvec3(R, zb, o);
    for (int r = 0; r < 3; ++r) o[r] += t[r];
    double A[21], g[6];
    for (int k = 0; k < 21; ++k) A[k] = 0;
    for (int k = 0; k < 6; ++k) g[k] = 0;
    for (int i = 0; i < n; ++i) {
      double m[3] = {Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]}, P[3];
      matvec3(R, m, P);
      for (int r = 0; r < 3; ++r) P[r] += t[r];
      if (!(P[2] > z_min)) return false;
      double iz = 1.0 / P[2];
      double u = Kd[0] * (P[0] * iz) + Kd[2], v = Kd[1] * (P[1] * iz) + Kd[3];
      double w[3];
      whiten_factor<double>(shapes + 4 * i, w);
      double r0 = (double)z[3 * i] - u, r1 = (double)z[3 * i + 1] - v;
      double rt0 = w[0] * r0 + w[1] * r1, rt1 = w[2] * r1;
      double pt[3] = {P[0] - o[0], P[1] - o[1], P[2] - o[2]};
      gn_accumulate<double>(P, pt, iz, Kd[0], Kd[1], w, rt0, rt1, A, g);
    }
    double d[6];
    if (!chol6_solve<double>(A, g, d)) return false;
    apply_update<double>(d, o, R, t);
  }
  for (int i = 0; i < n; ++i) {
    double m[3] = {Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]}, P[3];
    matvec3(R, m, P);
    if (!(P[2] + t[2] > z_min)) return false;
  }
  return true;
}

// Weighted cost sum ||z_i - Pi(R Z_i + t)||^2_Lambda_i of a 2D-3D pose.
__device__ double cost_2d(const float *Z, const float *z, const float *shapes, int n, const float K[4],
                          const double R[9], const double t[3]) {
  double c = 0;
  for (int i = 0; i < n; ++i) {
    double m[3] = {Z[3 * i], Z[3 * i + 1], Z[3 * i + 2]}, P[3];
    matvec3(R, m, P);
    for (int r = 0; r < 3; ++r) P[r] += t[r];
    double iz = 1.0 / P[2];
    double u = (double)K[0] * (P[0] * iz) + K[2], v = (double)K[1] * (P[1] * iz) + K[3];
    double w[3];
    whiten_factor<double>(shapes + 4 * i, w);
    double r0 = (double)z[3 * i] - u, r1 = (double)z[3 * i + 1] - v;
    double a = w[0] * r0 + w[1] * r1, b = w[2] * r1;
    c += a * a + b * b;
  }
  return c;
}

// Arun's method in float64: R = proj_SO3(sum (b_i - bbar)(a_i - abar)^T).
__device__ void kabsch_centre(const float *a, const float *b, int n, double R[9], double t[3]) {
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

}  // namespace

__global__ void __launch_bounds__(64) k_prologue(DevBatch b, DevParams p, InstRec *inst, KpRec *kprec,
                                                 int32_t *inst_status) {
  const int j = blockIdx.x;
  if (threadIdx.x != 0) return;
  InstRec I;
  I.kind = b.kind[j];
  I.n_kp = b.n_kp[j];
  I.kp_off = b.kp_off[j];
  int64_t soff, sM;
  sample_range(b.sample_off, j, b.total_samples, b.max_samples, soff, sM);
  I.sample_off = soff;
  I.n_samples = sM;
  const bool kp_ok = I.kp_off >= 0 && b.kp_off[j + 1] - I.kp_off == (int64_t)I.n_kp &&
                     b.kp_off[j + 1] <= b.total_kp;
  I.seed = b.seed[j];
  I.has_anchor = 0;
  I.status = PURSE_INST_OK;
  for (int k = 0; k < 4; ++k) I.K[k] = (I.kind == PURSE_KIND_2D3D) ? b.intrinsics[4 * j + k] : 0.f;
  for (int k = 0; k < 9; ++k) I.Rc[k] = I.Ra[k] = (k % 4 == 0) ? 1.f : 0.f;
  for (int k = 0; k < 3; ++k) I.tc[k] = I.ta[k] = I.oc[k] = I.abar[k] = 0.f;
  I.pad[0] = I.pad[1] = 0.f;
  const int n = I.n_kp;
  const bool is2d = I.kind == PURSE_KIND_2D3D;
  const int64_t ko = kp_ok ? I.kp_off : 0;
  const float *a = b.model_pts + 3 * ko;
  const float *c = b.centres + 3 * ko;
  const float *L = b.shapes + 4 * ko;
  const float *beta = b.bounds + ko;
  // ---- validation
  if ((I.kind != PURSE_KIND_3D3D && !is2d) || !kp_ok || n < (is2d ? 6 : 3) || n > PURSE_MAX_KP ||
      I.n_samples < 1 || n > b.max_kp) {
    I.status = PURSE_INST_BAD_SIZE;
  } else {
    bool good = true;
    for (int i = 0; i < n && good; ++i) {
      for (int r = 0; r < 3; ++r) good = good && finite_f(a[3 * i + r]);
      good = good && finite_f(c[3 * i]) && finite_f(c[3 * i + 1]) && (is2d || finite_f(c[3 * i + 2]));
      good = good && finite_f(beta[i]) && beta[i] >= 0.f;
      if (is2d) {
        const float *l = L + 4 * i;
        good = good && finite_f(l[0]) && finite_f(l[1]) && finite_f(l[2]) && finite_f(l[3]);
        good = good && l[1] == l[2] && l[0] > 0.f && (double)l[0] * l[3] - (double)l[1] * l[2] > 0.0;
      }
    }
    if (is2d)
      for (int k = 0; k < 4; ++k) good = good && finite_f(I.K[k]);
    if (is2d) good = good && I.K[0] > 0.f && I.K[1] > 0.f;
    if (!good) I.status = PURSE_INST_BAD_SHAPE;
  }
  if (I.status != PURSE_INST_OK) {
    inst[j] = I;
    inst_status[j] = I.status;
    return;
  }
  // ---- keypoint records
  double ab[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) ab[r] += a[3 * i + r];
  for (int r = 0; r < 3; ++r) ab[r] /= n;
  for (int r = 0; r < 3; ++r) I.abar[r] = (float)ab[r];
  const float tau = is2d ? p.tau2 : p.tau3;
  KpRec *kp = kprec + I.kp_off;
  for (int i = 0; i < n; ++i) {
    KpRec k;
    for (int r = 0; r < 3; ++r) {
      k.m[r] = is2d ? a[3 * i + r] : (float)((double)a[3 * i + r] - ab[r]);
      k.c[r] = (r < 2 || !is2d) ? c[3 * i + r] : 0.f;
      k.w[r] = 0.f;
    }
    if (is2d) {
      double w[3];
      whiten_factor<double>(L + 4 * i, w);
      for (int r = 0; r < 3; ++r) k.w[r] = (float)w[r];
    }
    k.kb = (float)((double)p.kappa * beta[i]);
    k.kb2 = k.kb * k.kb;
    k.bt = (float)((double)beta[i] + tau);
    kp[i] = k;
  }
  // ---- centre fit
  double Rd[9], td[3];
  bool fit_ok = true;
  if (is2d) {
    // Gauss-Newton from the DLT and from the weak-perspective fit; the
    // successful fit with the lower cost is kept (ties: the DLT one)
    double Ra_[9], ta_[3];
    bool ok1 = dlt_2d(a, c, n, I.K, Rd, td);
    if (ok1) ok1 = gn_centre_2d(a, c, L, n, I.K, p.centre_gn, (double)p.z_min, Rd, td);
    bool ok2 = affine_2d(a, c, n, I.K, Ra_, ta_);
    if (ok2) ok2 = gn_centre_2d(a, c, L, n, I.K, p.centre_gn, (double)p.z_min, Ra_, ta_);
    if (ok2 && (!ok1 || cost_2d(a, c, L, n, I.K, Ra_, ta_) < cost_2d(a, c, L, n, I.K, Rd, td))) {
      for (int k = 0; k < 9; ++k) Rd[k] = Ra_[k];
      for (int k = 0; k < 3; ++k) td[k] = ta_[k];
    }
    fit_ok = ok1 || ok2;
  } else {
    kabsch_centre(a, c, n, Rd, td);
  }
  for (int k = 0; k < 9; ++k) I.Rc[k] = (float)Rd[k];
  for (int r = 0; r < 3; ++r) I.tc[r] = (float)td[r];
  if (!fit_ok) {
    I.status = PURSE_INST_FIT_FAILED;
    inst[j] = I;
    inst_status[j] = I.status;
    return;
  }
  double oc[3];
  matvec3(Rd, ab, oc);
  for (int r = 0; r < 3; ++r) I.oc[r] = (float)(oc[r] + td[r]);
  // ---- anchor: x_c if inside the kappa-shrunk set, else the end of one
  // trajectory from x_c with no offset if that one is
  Pose xc;
  for (int k = 0; k < 9; ++k) xc.R[k] = I.Rc[k];
  for (int r = 0; r < 3; ++r) xc.t[r] = I.tc[r];
  bool inside = is2d ? feasible<PURSE_KIND_2D3D>(I, kp, xc, p, p.kappa)
                     : feasible<PURSE_KIND_3D3D>(I, kp, xc, p, p.kappa);
  if (inside) {
    I.has_anchor = 1;
    for (int k = 0; k < 9; ++k) I.Ra[k] = xc.R[k];
    for (int r = 0; r < 3; ++r) I.ta[r] = xc.t[r];
  } else {
    I.status |= PURSE_INST_ANCHOR_ITERATED;
    int nfb = 0;
    Pose x = xc;
    uint8_t m = is2d ? run_trajectory<PURSE_KIND_2D3D>(I, kp, x, p, false, nfb)
                     : run_trajectory<PURSE_KIND_3D3D>(I, kp, x, p, false, nfb);
    bool ok = (m & PURSE_MASK_FAILED) == 0;
    if (ok)
      ok = is2d ? feasible<PURSE_KIND_2D3D>(I, kp, x, p, p.kappa) : feasible<PURSE_KIND_3D3D>(I, kp, x, p, p.kappa);
    if (ok) {
      I.has_anchor = 1;
      for (int k = 0; k < 9; ++k) I.Ra[k] = x.R[k];
      for (int r = 0; r < 3; ++r) I.ta[r] = x.t[r];
    } else {
      I.status |= PURSE_INST_NO_ANCHOR;
    }
  }
  inst[j] = I;
  inst_status[j] = I.status;
}

void launch_prologue(const DevBatch &b, const DevParams &p, InstRec *inst, KpRec *kp, int32_t *inst_status,
                     hipStream_t stream) {
  hipLaunchKernelGGL(k_prologue, dim3(b.n_inst), dim3(64), 0, stream, b, p, inst, kp, inst_status);
}

}  // namespace purse
