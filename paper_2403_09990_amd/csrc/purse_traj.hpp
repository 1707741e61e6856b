// One PURSE trajectory per lane: initial offset, alternating iterations,
// feasibility test and bisection pull-in.  float32 throughout, except the
// float64 polar step taken when the float32 one is ill-conditioned.
#pragma once

#include "purse_device.hpp"

namespace purse {

struct Pose {
  float R[9];
  float t[3];
};

// Outward start of trajectory s: direction u on S^2 from two 24-bit Philox
// uniforms (z = 1 - 2 U1, phi = 2 pi U2); even s rotate the object about the
// pivot by omega0 u, odd s shift it by v0 u.
__device__ __forceinline__ Pose initial_pose(const InstRec &I, uint64_t s, const DevParams &p) {
  uint64_t c[4] = {s, 0ull, 0ull, 0ull};
  philox4x64_10(c, I.seed, 0ull);
  float u1 = (float)(c[0] >> 40) * 0x1p-24f;
  float u2 = (float)(c[1] >> 40) * 0x1p-24f;
  float z = 1.f - 2.f * u1;
  float rho = sqrtf(fmaxf(0.f, 1.f - z * z));
  float sp, cp;
  sincospif(2.f * u2, &sp, &cp);
  float d[3] = {rho * cp, rho * sp, z};
  Pose x;
  if ((s & 1ull) == 0ull) {
    float w[3] = {p.omega0 * d[0], p.omega0 * d[1], p.omega0 * d[2]};
    float E[9];
    exp_so3(w, E);
    matmul3(E, I.Rc, x.R);
    float r[3] = {I.tc[0] - I.oc[0], I.tc[1] - I.oc[1], I.tc[2] - I.oc[2]}, e[3];
    matvec3(E, r, e);
    x.t[0] = e[0] + I.oc[0];
    x.t[1] = e[1] + I.oc[1];
    x.t[2] = e[2] + I.oc[2];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) x.R[k] = I.Rc[k];
    x.t[0] = I.tc[0] + p.v0 * d[0];
    x.t[1] = I.tc[1] + p.v0 * d[1];
    x.t[2] = I.tc[2] + p.v0 * d[2];
  }
  return x;
}

// ---------------------------------------------------------------------------
// 3D-3D: project b_i + s_i e_i (ball of radius kappa beta_i), refit by Arun's
// method: R = proj_SO3(sum q_i (a_i - abar)^T), t = qbar - R abar.
__device__ __forceinline__ void polar_step(const float M[9], float R[9], bool force64, int &n_fb) {
  bool ok = false;
  if (!force64) ok = polar_so3<float>(M, R, 4);
  if (!ok) {
    double Md[9], Rd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Md[k] = (double)M[k];
    polar_so3<double>(Md, Rd, 10);
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (float)Rd[k];
    ++n_fb;
  }
}

__device__ __forceinline__ void traj3d(const KpRec *__restrict__ kp, int n, const float abar[3],
                                       int n_iters, bool force64, Pose &x, int &n_fb) {
  const float inv_n = 1.f / (float)n;
  for (int it = 0; it < n_iters; ++it) {
    float tt[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      tt[r] = x.t[r] + x.R[3 * r] * abar[0] + x.R[3 * r + 1] * abar[1] + x.R[3 * r + 2] * abar[2];
    float M[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float qs[3] = {0.f, 0.f, 0.f};
    // targets are accumulated relative to the predicted centroid tt, so the
    // float32 rounding of sum(a_i - abar) = 0 cannot leak a large q_bar into M
    for (int i = 0; i < n; ++i) {
      const KpRec k = kp[i];
      float d[3], e[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        d[r] = tt[r] - k.c[r];
        e[r] = x.R[3 * r] * k.m[0] + x.R[3 * r + 1] * k.m[1] + x.R[3 * r + 2] * k.m[2] + d[r];
      }
      float r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
      float s = (r2 <= k.kb2) ? 1.f : k.kb * rsqrtf(r2);
      float q[3] = {s * e[0] - d[0], s * e[1] - d[1], s * e[2] - d[2]};  // q_i - tt
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        M[3 * r] += q[r] * k.m[0];
        M[3 * r + 1] += q[r] * k.m[1];
        M[3 * r + 2] += q[r] * k.m[2];
        qs[r] += q[r];
      }
    }
    polar_step(M, x.R, force64, n_fb);
    float ra[3];
    matvec3(x.R, abar, ra);
    x.t[0] = tt[0] + qs[0] * inv_n - ra[0];
    x.t[1] = tt[1] + qs[1] * inv_n - ra[1];
    x.t[2] = tt[2] + qs[2] * inv_n - ra[2];
  }
}

__device__ __forceinline__ bool feasible3d(const KpRec *__restrict__ kp, int n, const float abar[3],
                                           const Pose &x, float margin_k) {
  // margin_k < 0: test r_i <= beta_i + tau; else r_i <= kappa beta_i + tau
  float tt[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    tt[r] = x.t[r] + x.R[3 * r] * abar[0] + x.R[3 * r + 1] * abar[1] + x.R[3 * r + 2] * abar[2];
  bool ok = true;
  for (int i = 0; i < n; ++i) {
    const KpRec k = kp[i];
    float e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      e[r] = x.R[3 * r] * k.m[0] + x.R[3 * r + 1] * k.m[1] + x.R[3 * r + 2] * k.m[2] + tt[r] - k.c[r];
    float rr = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    float bound = margin_k < 0.f ? k.bt : k.kb + (k.bt - k.kb / margin_k);
    ok = ok && (rr <= bound);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// 2D-3D: project z_i + s_i e_i (ellipse shrunk by kappa, radial in the
// Lambda metric), refit by n_gn Gauss-Newton steps about the pivot.  The
// first step evaluates at the projection pose, where q - u = (s - 1) e; later
// steps recompute the targets from the saved projection pose.
__device__ __forceinline__ void project2d(const float R[9], const float t[3], const KpRec &k,
                                          const float K[4], float P[3], float &iz, float &u, float &v) {
#pragma unroll
  for (int r = 0; r < 3; ++r) P[r] = R[3 * r] * k.m[0] + R[3 * r + 1] * k.m[1] + R[3 * r + 2] * k.m[2] + t[r];
  iz = 1.f / P[2];
  u = K[0] * (P[0] * iz) + K[2];
  v = K[1] * (P[1] * iz) + K[3];
}

__device__ __forceinline__ bool traj2d(const KpRec *__restrict__ kp, int n, const float K[4],
                                       const float oc[3], int n_iters, int n_gn, float z_min, Pose &x) {
  for (int it = 0; it < n_iters; ++it) {
    const Pose xk = x;
    for (int gs = 0; gs < n_gn; ++gs) {
      float A[21], g[6];
#pragma unroll
      for (int k = 0; k < 21; ++k) A[k] = 0.f;
#pragma unroll
      for (int k = 0; k < 6; ++k) g[k] = 0.f;
      bool ok = true;
      for (int i = 0; i < n; ++i) {
        const KpRec k = kp[i];
        float P[3], iz, u, v;
        project2d(x.R, x.t, k, K, P, iz, u, v);
        ok = ok && (P[2] > z_min);
        float rt0, rt1;
        if (gs == 0) {
          float e0 = u - k.c[0], e1 = v - k.c[1];
          float et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
          float r2 = et0 * et0 + et1 * et1;
          float s = (r2 <= k.kb2) ? 1.f : k.kb * rsqrtf(r2);
          rt0 = (s - 1.f) * et0;
          rt1 = (s - 1.f) * et1;
        } else {
          float Pk[3], izk, uk, vk;
          project2d(xk.R, xk.t, k, K, Pk, izk, uk, vk);
          float e0 = uk - k.c[0], e1 = vk - k.c[1];
          float et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
          float r2 = et0 * et0 + et1 * et1;
          float s = (r2 <= k.kb2) ? 1.f : k.kb * rsqrtf(r2);
          float r0 = k.c[0] + s * e0 - u, r1 = k.c[1] + s * e1 - v;
          rt0 = k.w[0] * r0 + k.w[1] * r1;
          rt1 = k.w[2] * r1;
        }
        float pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
        gn_accumulate<float>(P, pt, iz, K[0], K[1], k.w, rt0, rt1, A, g);
      }
      float d[6];
      ok = ok && chol6_solve<float>(A, g, d);
      if (!ok) return false;
      apply_update<float>(d, oc, x.R, x.t);
    }
  }
  return true;
}

__device__ __forceinline__ bool feasible2d(const KpRec *__restrict__ kp, int n, const float K[4],
                                           const Pose &x, float z_min, float margin_k) {
  bool ok = true;
  for (int i = 0; i < n; ++i) {
    const KpRec k = kp[i];
    float P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    float e0 = u - k.c[0], e1 = v - k.c[1];
    float et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
    float rr = sqrtf(et0 * et0 + et1 * et1);
    float bound = margin_k < 0.f ? k.bt : k.kb + (k.bt - k.kb / margin_k);
    ok = ok && (P[2] > z_min) && (rr <= bound);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// One Bjorck step R <- R (3 I - R^T R) / 2 removes the float32 drift from
// orthonormality accumulated over many left updates.
__device__ __forceinline__ void reorthonormalise(float R[9]) {
  float S[9], Q[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S[3 * r + c] = -(R[r] * R[c] + R[3 + r] * R[3 + c] + R[6 + r] * R[6 + c]);
  S[0] += 3.f;
  S[4] += 3.f;
  S[8] += 3.f;
  matmul3(R, S, Q);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = 0.5f * Q[k];
}

template <int KIND>
__device__ __forceinline__ bool feasible(const InstRec &I, const KpRec *__restrict__ kp, const Pose &x,
                                         const DevParams &p, float margin_k) {
  if (KIND == PURSE_KIND_3D3D) return feasible3d(kp, I.n_kp, I.abar, x, margin_k);
  return feasible2d(kp, I.n_kp, I.K, x, p.z_min, margin_k);
}

// Bisection on x(l) = (R_a Exp(l Log(R_a^T R)), t_a + l (t - t_a)) between the
// feasible anchor (l = 0) and the infeasible end (l = 1); keeps the feasible end.
template <int KIND>
__device__ __forceinline__ Pose pull_in(const InstRec &I, const KpRec *__restrict__ kp, const Pose &x,
                                        const DevParams &p) {
  float RtR[9], RaT[9], w[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) RaT[3 * r + c] = I.Ra[3 * c + r];
  matmul3(RaT, x.R, RtR);
  log_so3(RtR, w);
  float lo = 0.f, hi = 1.f;
  for (int b = 0; b < p.n_bis; ++b) {
    float mid = 0.5f * (lo + hi);
    float wm[3] = {mid * w[0], mid * w[1], mid * w[2]}, E[9];
    Pose m;
    exp_so3(wm, E);
    matmul3(I.Ra, E, m.R);
#pragma unroll
    for (int r = 0; r < 3; ++r) m.t[r] = I.ta[r] + mid * (x.t[r] - I.ta[r]);
    if (feasible<KIND>(I, kp, m, p, -1.f))
      lo = mid;
    else
      hi = mid;
  }
  Pose out;
  if (lo == 0.f) {
#pragma unroll
    for (int k = 0; k < 9; ++k) out.R[k] = I.Ra[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) out.t[r] = I.ta[r];
  } else {
    float wl[3] = {lo * w[0], lo * w[1], lo * w[2]}, E[9];
    exp_so3(wl, E);
    matmul3(I.Ra, E, out.R);
#pragma unroll
    for (int r = 0; r < 3; ++r) out.t[r] = I.ta[r] + lo * (x.t[r] - I.ta[r]);
  }
  return out;
}

// Full trajectory from x; returns the mask bits and leaves the output pose in x.
template <int KIND>
__device__ __forceinline__ uint8_t run_trajectory(const InstRec &I, const KpRec *__restrict__ kp, Pose &x,
                                                  const DevParams &p, bool with_pull_in, int &n_fb) {
  bool ok = true;
  if (KIND == PURSE_KIND_3D3D) {
    traj3d(kp, I.n_kp, I.abar, p.n_iters, (p.flags & PURSE_FLAG_FORCE_FP64_POLAR) != 0, x, n_fb);
  } else {
    ok = traj2d(kp, I.n_kp, I.K, I.oc, p.n_iters, p.n_gn, p.z_min, x);
    reorthonormalise(x.R);
  }
  if (!ok) return PURSE_MASK_FAILED;
  if (feasible<KIND>(I, kp, x, p, -1.f)) return PURSE_MASK_FEASIBLE;
  if (with_pull_in && I.has_anchor) {
    x = pull_in<KIND>(I, kp, x, p);
    return PURSE_MASK_FEASIBLE | PURSE_MASK_PULLED_IN;
  }
  return 0;
}

}  // namespace purse
