// One PURSE trajectory per lane: initial offset, alternating iterations,
// feasibility test and bisection pull-in.  Written once over the scalar type
// T: float for the sampler (float64 only in the ill-conditioned polar step),
// Dual<float> when the backward re-runs a trajectory to get its tangent along
// one input direction.
#pragma once

#include "purse_device.hpp"

namespace purse {

template <typename T>
struct PoseT {
  T R[9];
  T t[3];
};
using Pose = PoseT<float>;

// Per-instance frame of a trajectory: centre x_c, pivot o_c, anchor x_a.
template <typename T>
struct FrameT {
  T Rc[9], tc[3], oc[3], Ra[9], ta[3];
};

// A keypoint as the trajectory sees it: model point (never differentiated)
// and the constraint data (centre, whitening, kappa beta, (kappa beta)^2,
// beta + tau), which carry tangents in the backward.
template <typename T>
struct KpT {
  float m[3];
  T c[3], w[3], kb, kb2, bt;
};

// Keypoint loader of the sampler: the prologue's records as they are.  The
// records are uniform across the workgroup, so they live in scalar registers;
// kPrefetch asks the loops to fetch record i + 1 while record i is in use.
struct KpPlain {
  static constexpr bool kPrefetch = true;
  const KpRec *__restrict__ kp;
  __device__ __forceinline__ KpRec operator()(int i) const { return kp[i]; }
};

// Sequential reader over keypoints 0..n-1 of a loader, one record ahead when
// the loader asks for it (the load latency then overlaps a keypoint's work).
template <typename KPL>
struct KpSeq {
  using Rec = decltype(((const KPL *)nullptr)->operator()(0));
  const KPL &kpl;
  int n;
  Rec nxt;
  __device__ __forceinline__ KpSeq(const KPL &l, int n_) : kpl(l), n(n_) {
    if constexpr (KPL::kPrefetch) nxt = kpl(0);
  }
  __device__ __forceinline__ Rec operator()(int i) {
    if constexpr (KPL::kPrefetch) {
      Rec k = nxt;
      nxt = kpl(i + 1 < n ? i + 1 : i);
      return k;
    } else {
      return kpl(i);
    }
  }
};

// Clamp threshold on r^2 / (kappa beta)^2.  Derivatives treat a constraint
// within a relative 1e-5 inside its shrunk ball as projected: converged
// trajectories end on that kink to rounding, approaching it from outside.
template <typename T> struct ClampBand { static constexpr float v = 1.0f; };
template <typename T> struct ClampBand<Dual<T>> { static constexpr float v = (1.0f - 1e-5f) * (1.0f - 1e-5f); };

// The frame read in place from the instance record (the sampler): each use
// is a load next to it, so the record does not hold registers across the
// whole trajectory.
struct FrameRef {
  const float *Rc, *tc, *oc, *Ra, *ta;
};

__device__ __forceinline__ FrameRef frame_ref(const InstRec &I) { return FrameRef{I.Rc, I.tc, I.oc, I.Ra, I.ta}; }

template <typename T>
__device__ __forceinline__ FrameT<T> frame_of(const InstRec &I) {
  FrameT<T> F;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F.Rc[k] = T(I.Rc[k]);
    F.Ra[k] = T(I.Ra[k]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    F.tc[r] = T(I.tc[r]);
    F.oc[r] = T(I.oc[r]);
    F.ta[r] = T(I.ta[r]);
  }
  return F;
}

// Outward start of trajectory s: direction u on S^2 from two 24-bit Philox
// uniforms (z = 1 - 2 U1, phi = 2 pi U2); even s rotate the object about the
// pivot by omega0 u, odd s shift it by v0 u.
__device__ __forceinline__ void trajectory_direction(uint64_t seed, uint64_t s, float d[3]) {
  uint64_t c[4] = {s, 0ull, 0ull, 0ull};
  philox4x64_10(c, seed, 0ull);
  float u1 = (float)(c[0] >> 40) * 0x1p-24f;
  float u2 = (float)(c[1] >> 40) * 0x1p-24f;
  float z = 1.f - 2.f * u1;
  float rho = sqrtf(fmaxf(0.f, 1.f - z * z));
  float sp, cp;
  sincospif(2.f * u2, &sp, &cp);
  d[0] = rho * cp;
  d[1] = rho * sp;
  d[2] = z;
}

template <typename T, typename FR>
__device__ __forceinline__ PoseT<T> initial_pose(const FR &F, uint64_t seed, uint64_t s, const DevParams &p) {
  float d[3];
  trajectory_direction(seed, s, d);
  PoseT<T> x;
  if ((s & 1ull) == 0ull) {
    T w[3] = {T(p.omega0 * d[0]), T(p.omega0 * d[1]), T(p.omega0 * d[2])};
    T E[9];
    exp_so3(w, E);
    T Rc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Rc[k] = T(F.Rc[k]);
    matmul3(E, Rc, x.R);
    T r[3] = {T(F.tc[0]) - T(F.oc[0]), T(F.tc[1]) - T(F.oc[1]), T(F.tc[2]) - T(F.oc[2])}, e[3];
    matvec3(E, r, e);
#pragma unroll
    for (int k = 0; k < 3; ++k) x.t[k] = e[k] + T(F.oc[k]);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) x.R[k] = T(F.Rc[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) x.t[k] = T(F.tc[k]) + T(p.v0 * d[k]);
  }
  return x;
}

// ---------------------------------------------------------------------------
// 3D-3D: project b_i + s_i e_i (ball of radius kappa beta_i), refit by Arun's
// method: R = proj_SO3(sum (q_i - tt) (a_i - abar)^T), t = qbar - R abar.
__device__ __forceinline__ void polar_fp64(const float M[9], float R[9]) {
  double Md[9], Rd[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Md[k] = (double)M[k];
  polar_so3<double>(Md, Rd, 10);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = (float)Rd[k];
}

template <typename T>
__device__ __forceinline__ void polar_fp64(const Dual<T> M[9], Dual<T> R[9]) {
  Dual<double> Md[9], Rd[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Md[k] = Dual<double>((double)M[k].v, (double)M[k].d);
  polar_so3<Dual<double>>(Md, Rd, 10);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = Dual<T>((T)Rd[k].v, (T)Rd[k].d);
}

template <typename T>
__device__ __forceinline__ void polar_step(const T M[9], T R[9], bool force64, int &n_fb) {
  bool ok = false;
  if (!force64) ok = polar_so3<T>(M, R, 4);
  if (!ok) {
    polar_fp64(M, R);
    ++n_fb;
  }
}

template <typename T, typename KPL>
__device__ __forceinline__ void traj3d(const KPL &kpl, int n, const float abar[3], int n_iters, bool force64,
                                       PoseT<T> &x, int &n_fb) {
  const float inv_n = 1.f / (float)n;
  const float band = ClampBand<T>::v;
  for (int it = 0; it < n_iters; ++it) {
    T tt[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      tt[r] = x.t[r] + x.R[3 * r] * abar[0] + x.R[3 * r + 1] * abar[1] + x.R[3 * r + 2] * abar[2];
    T M[9], qs[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = T(0.f);
#pragma unroll
    for (int k = 0; k < 3; ++k) qs[k] = T(0.f);
    // targets are accumulated relative to the predicted centroid tt, so the
    // float32 rounding of sum(a_i - abar) = 0 cannot leak a large q_bar into M
    KpSeq<KPL> seq(kpl, n);
    for (int i = 0; i < n; ++i) {
      const auto k = seq(i);
      T d[3], e[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        d[r] = tt[r] - k.c[r];
        e[r] = x.R[3 * r] * k.m[0] + x.R[3 * r + 1] * k.m[1] + x.R[3 * r + 2] * k.m[2] + d[r];
      }
      T r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
      T s = (r2 <= k.kb2 * band) ? T(1.f) : k.kb * drsqrt(r2);
      T q[3] = {s * e[0] - d[0], s * e[1] - d[1], s * e[2] - d[2]};  // q_i - tt
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        M[3 * r] += q[r] * k.m[0];
        M[3 * r + 1] += q[r] * k.m[1];
        M[3 * r + 2] += q[r] * k.m[2];
        qs[r] += q[r];
      }
    }
    polar_step(M, x.R, force64, n_fb);
    T ra[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) ra[r] = x.R[3 * r] * abar[0] + x.R[3 * r + 1] * abar[1] + x.R[3 * r + 2] * abar[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) x.t[r] = tt[r] + qs[r] * inv_n - ra[r];
  }
}

// margin_k < 0: test r_i <= beta_i + tau; else r_i <= kappa beta_i + tau
template <typename T, typename KPL>
__device__ __forceinline__ bool feasible3d(const KPL &kpl, int n, const float abar[3], const PoseT<T> &x,
                                           float margin_k) {
  T tt[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    tt[r] = x.t[r] + x.R[3 * r] * abar[0] + x.R[3 * r + 1] * abar[1] + x.R[3 * r + 2] * abar[2];
  bool ok = true;
  for (int i = 0; i < n; ++i) {
    const auto k = kpl(i);
    T e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      e[r] = x.R[3 * r] * k.m[0] + x.R[3 * r + 1] * k.m[1] + x.R[3 * r + 2] * k.m[2] + tt[r] - k.c[r];
    float rr = sqrtf(value_of(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
    float kb = value_of(k.kb), bt = value_of(k.bt);
    float bound = margin_k < 0.f ? bt : kb + (bt - kb / margin_k);
    ok = ok && (rr <= bound);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// 2D-3D: project z_i + s_i e_i (ellipse shrunk by kappa, radial in the
// Lambda metric), refit by n_gn Gauss-Newton steps about the pivot.  The
// first step evaluates at the projection pose, where q - u = (s - 1) e; later
// steps recompute the targets from the saved projection pose.
template <typename T, typename KK>
__device__ __forceinline__ void project2d(const T R[9], const T t[3], const KK &k, const float K[4], T P[3],
                                          T &iz, T &u, T &v) {
#pragma unroll
  for (int r = 0; r < 3; ++r) P[r] = R[3 * r] * k.m[0] + R[3 * r + 1] * k.m[1] + R[3 * r + 2] * k.m[2] + t[r];
  iz = drcp(P[2]);
  u = K[0] * (P[0] * iz) + K[2];
  v = K[1] * (P[1] * iz) + K[3];
}

// One Gauss-Newton step of the 2D-3D refit from x towards the targets of the
// projection pose xk (FIRST: x == xk, so the residual is (s - 1) e).
template <bool FIRST, typename T, typename KPL>
__device__ __forceinline__ bool gn_pass2d(const KPL &kpl, int n, const float K[4], const T oc[3], float z_min,
                                          float band, const PoseT<T> &xk, PoseT<T> &x) {
  T A[21], g[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = T(0.f);
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = T(0.f);
  bool ok = true;
  KpSeq<KPL> seq(kpl, n);
  for (int i = 0; i < n; ++i) {
    const auto k = seq(i);
    T P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    ok = ok && (P[2] > z_min);
    T rt0, rt1;
    if (FIRST) {
      T e0 = u - k.c[0], e1 = v - k.c[1];
      T et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
      T r2 = et0 * et0 + et1 * et1;
      T s = (r2 <= k.kb2 * band) ? T(1.f) : k.kb * drsqrt(r2);
      rt0 = (s - 1.f) * et0;
      rt1 = (s - 1.f) * et1;
    } else {
      T Pk[3], izk, uk, vk;
      project2d(xk.R, xk.t, k, K, Pk, izk, uk, vk);
      T e0 = uk - k.c[0], e1 = vk - k.c[1];
      T et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
      T r2 = et0 * et0 + et1 * et1;
      T s = (r2 <= k.kb2 * band) ? T(1.f) : k.kb * drsqrt(r2);
      T r0 = k.c[0] + s * e0 - u, r1 = k.c[1] + s * e1 - v;
      rt0 = k.w[0] * r0 + k.w[1] * r1;
      rt1 = k.w[2] * r1;
    }
    T pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
    gn_accumulate<T>(P, pt, iz, T(K[0]), T(K[1]), k.w, rt0, rt1, A, g);
  }
  T d[6];
  ok = ok && chol6_solve<T>(A, g, d);
  if (!ok) return false;
  apply_update<T>(d, oc, x.R, x.t);
  return true;
}

// The same Gauss-Newton step with the keypoint loop unrolled for at most NMAX
// keypoints and the projection targets of the current iteration held in
// registers: the first step computes q_i = c_i + s_i e_i at xk and keeps it,
// later steps only re-project at x.  Arithmetic as in gn_pass2d.
template <bool FIRST, int NMAX, typename T, typename KPL>
__device__ __forceinline__ bool gn_pass2d_unrolled(const KPL &kpl, int n, const float K[4], const T oc[3],
                                                   float z_min, float band, T tq[NMAX][2], PoseT<T> &x) {
  T A[21], g[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = T(0.f);
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = T(0.f);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    if (i < n) {
      const auto k = kpl(i);
      T P[3], iz, u, v;
      project2d(x.R, x.t, k, K, P, iz, u, v);
      ok = ok && (P[2] > z_min);
      T rt0, rt1;
      if (FIRST) {
        T e0 = u - k.c[0], e1 = v - k.c[1];
        T et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
        T r2 = et0 * et0 + et1 * et1;
        T s = (r2 <= k.kb2 * band) ? T(1.f) : k.kb * drsqrt(r2);
        rt0 = (s - 1.f) * et0;
        rt1 = (s - 1.f) * et1;
        tq[i][0] = k.c[0] + s * e0;
        tq[i][1] = k.c[1] + s * e1;
      } else {
        T r0 = tq[i][0] - u, r1 = tq[i][1] - v;
        rt0 = k.w[0] * r0 + k.w[1] * r1;
        rt1 = k.w[2] * r1;
      }
      T pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
      gn_accumulate<T>(P, pt, iz, T(K[0]), T(K[1]), k.w, rt0, rt1, A, g);
    }
  }
  T d[6];
  ok = ok && chol6_solve<T>(A, g, d);
  if (!ok) return false;
  apply_update<T>(d, oc, x.R, x.t);
  return true;
}

// NMAX > 0: at most NMAX keypoints, loops unrolled (gn_pass2d_unrolled).
template <int NMAX, typename T, typename KPL>
__device__ __forceinline__ bool traj2d(const KPL &kpl, int n, const float K[4], const T oc[3], int n_iters,
                                       int n_gn, float z_min, PoseT<T> &x) {
  const float band = ClampBand<T>::v;
  for (int it = 0; it < n_iters; ++it) {
    if constexpr (NMAX > 0) {
      T tq[NMAX][2];
      if (!gn_pass2d_unrolled<true, NMAX>(kpl, n, K, oc, z_min, band, tq, x)) return false;
      for (int gs = 1; gs < n_gn; ++gs)
        if (!gn_pass2d_unrolled<false, NMAX>(kpl, n, K, oc, z_min, band, tq, x)) return false;
    } else {
      const PoseT<T> xk = x;
      if (!gn_pass2d<true>(kpl, n, K, oc, z_min, band, xk, x)) return false;
      for (int gs = 1; gs < n_gn; ++gs)
        if (!gn_pass2d<false>(kpl, n, K, oc, z_min, band, xk, x)) return false;
    }
  }
  return true;
}

template <typename T, typename KPL>
__device__ __forceinline__ bool feasible2d(const KPL &kpl, int n, const float K[4], const PoseT<T> &x,
                                           float z_min, float margin_k) {
  bool ok = true;
  for (int i = 0; i < n; ++i) {
    const auto k = kpl(i);
    T P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    T e0 = u - k.c[0], e1 = v - k.c[1];
    T et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
    float rr = sqrtf(value_of(et0 * et0 + et1 * et1));
    float kb = value_of(k.kb), bt = value_of(k.bt);
    float bound = margin_k < 0.f ? bt : kb + (bt - kb / margin_k);
    ok = ok && (value_of(P[2]) > z_min) && (rr <= bound);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// One Bjorck step R <- R (3 I - R^T R) / 2 removes the float32 drift from
// orthonormality accumulated over many left updates.
template <typename T>
__device__ __forceinline__ void reorthonormalise(T R[9]) {
  T S[9], Q[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S[3 * r + c] = -(R[r] * R[c] + R[3 + r] * R[3 + c] + R[6 + r] * R[6 + c]);
  S[0] += T(3.f);
  S[4] += T(3.f);
  S[8] += T(3.f);
  matmul3(R, S, Q);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = T(0.5f) * Q[k];
}

template <int KIND, typename T, typename KPL>
__device__ __forceinline__ bool feasible(const InstRec &I, const KPL &kpl, const PoseT<T> &x, const DevParams &p,
                                         float margin_k) {
  if (KIND == PURSE_KIND_3D3D) return feasible3d(kpl, I.n_kp, I.abar, x, margin_k);
  return feasible2d(kpl, I.n_kp, I.K, x, p.z_min, margin_k);
}

// Bisection on x(l) = (R_a Exp(l Log(R_a^T R)), t_a + l (t - t_a)) between the
// feasible anchor (l = 0) and the infeasible end (l = 1); keeps the feasible end.
template <int KIND, typename T, typename KPL, typename FR>
__device__ __forceinline__ PoseT<T> pull_in(const InstRec &I, const FR &F, const KPL &kpl, const PoseT<T> &x,
                                            const DevParams &p) {
  T Ra[9], ta[3], RtR[9], RaT[9], w[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ra[k] = T(F.Ra[k]);
#pragma unroll
  for (int r = 0; r < 3; ++r) ta[r] = T(F.ta[r]);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) RaT[3 * r + c] = Ra[3 * c + r];
  matmul3(RaT, x.R, RtR);
  log_so3(RtR, w);
  float lo = 0.f, hi = 1.f;
  for (int b = 0; b < p.n_bis; ++b) {
    float mid = 0.5f * (lo + hi);
    T wm[3] = {mid * w[0], mid * w[1], mid * w[2]}, E[9];
    PoseT<T> m;
    exp_so3(wm, E);
    matmul3(Ra, E, m.R);
#pragma unroll
    for (int r = 0; r < 3; ++r) m.t[r] = ta[r] + mid * (x.t[r] - ta[r]);
    if (feasible<KIND>(I, kpl, m, p, -1.f))
      lo = mid;
    else
      hi = mid;
  }
  PoseT<T> out;
  if (lo == 0.f) {
#pragma unroll
    for (int k = 0; k < 9; ++k) out.R[k] = Ra[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) out.t[r] = ta[r];
  } else {
    T wl[3] = {lo * w[0], lo * w[1], lo * w[2]}, E[9];
    exp_so3(wl, E);
    matmul3(Ra, E, out.R);
#pragma unroll
    for (int r = 0; r < 3; ++r) out.t[r] = ta[r] + lo * (x.t[r] - ta[r]);
  }
  return out;
}

// Full trajectory from x; returns the mask bits and leaves the output pose in x.
template <int KIND, int NMAX = 0, typename T, typename KPL, typename FR>
__device__ __forceinline__ uint8_t run_trajectory(const InstRec &I, const FR &F, const KPL &kpl,
                                                  PoseT<T> &x, const DevParams &p, bool with_pull_in,
                                                  int &n_fb) {
  bool ok = true;
  if (KIND == PURSE_KIND_3D3D) {
    traj3d(kpl, I.n_kp, I.abar, p.n_iters, (p.flags & PURSE_FLAG_FORCE_FP64_POLAR) != 0, x, n_fb);
  } else {
    T oc[3] = {T(F.oc[0]), T(F.oc[1]), T(F.oc[2])};
    ok = traj2d<NMAX>(kpl, I.n_kp, I.K, oc, p.n_iters, p.n_gn, p.z_min, x);
    reorthonormalise(x.R);
  }
  if (!ok) return PURSE_MASK_FAILED;
  if (feasible<KIND>(I, kpl, x, p, -1.f)) return PURSE_MASK_FEASIBLE;
  if (with_pull_in && I.has_anchor) {
    x = pull_in<KIND>(I, F, kpl, x, p);
    return PURSE_MASK_FEASIBLE | PURSE_MASK_PULLED_IN;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Lane-group modes (2D-3D, at most NMAX keypoints): G = 2 or 4 adjacent lanes
// of a wavefront run one trajectory together.  Lane q of the group takes the
// keypoints i = q, q + G, ...; the normal equations (and the feasibility and
// depth tests) are combined across the group by DPP quad permutations
// (butterfly sums), so every lane then holds the same sums (addition commutes)
// and computes the same step.  This divides the keypoint work per lane by G
// and multiplies the wavefronts of a batch by G.  Keypoint records come from
// LDS, where each lane reads its own.
template <int G>
__device__ __forceinline__ float lanes_sum(float x) {
  static_assert(G == 2 || G == 4, "groups within a quad");
  x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
  if (G == 4) x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  return x;
}

template <int G>
__device__ __forceinline__ bool lanes_and(bool b) {
  int v = b ? 1 : 0;
  v &= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  if (G == 4) v &= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  return v != 0;
}

template <bool FIRST, int NMAX, int G>
__device__ __forceinline__ bool gn_pass2d_lanes(const KpRec *kp, int n, int q, const float K[4], const float oc[3],
                                                float z_min, float tq[NMAX / G][2], Pose &x) {
  float A[21], g[6];
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = 0.f;
  bool ok = true;
#pragma unroll
  for (int ii = 0; ii < NMAX / G; ++ii) {
    const int i = G * ii + q;
    if (i < n) {
      const KpRec k = kp[i];
      float P[3], iz, u, v;
      project2d(x.R, x.t, k, K, P, iz, u, v);
      ok = ok && (P[2] > z_min);
      float rt0, rt1;
      if (FIRST) {
        float e0 = u - k.c[0], e1 = v - k.c[1];
        float et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
        float r2 = et0 * et0 + et1 * et1;
        float sc = (r2 <= k.kb2) ? 1.f : k.kb * drsqrt(r2);
        rt0 = (sc - 1.f) * et0;
        rt1 = (sc - 1.f) * et1;
        tq[ii][0] = k.c[0] + sc * e0;
        tq[ii][1] = k.c[1] + sc * e1;
      } else {
        float r0 = tq[ii][0] - u, r1 = tq[ii][1] - v;
        rt0 = k.w[0] * r0 + k.w[1] * r1;
        rt1 = k.w[2] * r1;
      }
      float pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
      gn_accumulate<float>(P, pt, iz, K[0], K[1], k.w, rt0, rt1, A, g);
    }
  }
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = lanes_sum<G>(A[k]);
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = lanes_sum<G>(g[k]);
  ok = lanes_and<G>(ok);
  float d[6];
  ok = ok && chol6_solve<float>(A, g, d);
  if (!ok) return false;
  apply_update<float>(d, oc, x.R, x.t);
  return true;
}

template <int NMAX, int G>
__device__ __forceinline__ bool traj2d_lanes(const KpRec *kp, int n, int q, const float K[4], const float oc[3],
                                             int n_iters, int n_gn, float z_min, Pose &x) {
  for (int it = 0; it < n_iters; ++it) {
    float tq[NMAX / G][2];
    if (!gn_pass2d_lanes<true, NMAX, G>(kp, n, q, K, oc, z_min, tq, x)) return false;
    for (int gs = 1; gs < n_gn; ++gs)
      if (!gn_pass2d_lanes<false, NMAX, G>(kp, n, q, K, oc, z_min, tq, x)) return false;
  }
  return true;
}

template <int NMAX, int G>
__device__ __forceinline__ bool feasible2d_lanes(const KpRec *kp, int n, int q, const float K[4], const Pose &x,
                                                 float z_min) {
  bool ok = true;
#pragma unroll
  for (int ii = 0; ii < NMAX / G; ++ii) {
    const int i = G * ii + q;
    if (i < n) {
      const KpRec k = kp[i];
      float P[3], iz, u, v;
      project2d(x.R, x.t, k, K, P, iz, u, v);
      float e0 = u - k.c[0], e1 = v - k.c[1];
      float et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
      ok = ok && (P[2] > z_min) && (sqrtf(et0 * et0 + et1 * et1) <= k.bt);
    }
  }
  return lanes_and<G>(ok);
}

// Lane-group trajectory: iterations, feasibility test, bisection pull-in.
template <int NMAX, int G>
__device__ __forceinline__ uint8_t run_trajectory_lanes(const InstRec &I, const FrameRef &F, const KpRec *kp, int q,
                                                        Pose &x, const DevParams &p) {
  const float oc[3] = {F.oc[0], F.oc[1], F.oc[2]};
  const bool ok = traj2d_lanes<NMAX, G>(kp, I.n_kp, q, I.K, oc, p.n_iters, p.n_gn, p.z_min, x);
  reorthonormalise(x.R);
  if (!ok) return PURSE_MASK_FAILED;
  if (feasible2d_lanes<NMAX, G>(kp, I.n_kp, q, I.K, x, p.z_min)) return PURSE_MASK_FEASIBLE;
  if (!I.has_anchor) return 0;
  float Ra[9], ta[3], RtR[9], RaT[9], w[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Ra[k] = F.Ra[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) ta[r] = F.ta[r];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) RaT[3 * r + c] = Ra[3 * c + r];
  matmul3(RaT, x.R, RtR);
  log_so3(RtR, w);
  float lo = 0.f, hi = 1.f;
  for (int b = 0; b < p.n_bis; ++b) {
    float mid = 0.5f * (lo + hi);
    float wm[3] = {mid * w[0], mid * w[1], mid * w[2]}, E[9];
    Pose m;
    exp_so3(wm, E);
    matmul3(Ra, E, m.R);
#pragma unroll
    for (int r = 0; r < 3; ++r) m.t[r] = ta[r] + mid * (x.t[r] - ta[r]);
    if (feasible2d_lanes<NMAX, G>(kp, I.n_kp, q, I.K, m, p.z_min))
      lo = mid;
    else
      hi = mid;
  }
  if (lo == 0.f) {
#pragma unroll
    for (int k = 0; k < 9; ++k) x.R[k] = Ra[k];
#pragma unroll
    for (int r = 0; r < 3; ++r) x.t[r] = ta[r];
  } else {
    float wl[3] = {lo * w[0], lo * w[1], lo * w[2]}, E[9];
    exp_so3(wl, E);
    matmul3(Ra, E, x.R);
#pragma unroll
    for (int r = 0; r < 3; ++r) x.t[r] = ta[r] + lo * (x.t[r] - ta[r]);
  }
  return PURSE_MASK_FEASIBLE | PURSE_MASK_PULLED_IN;
}

}  // namespace purse
