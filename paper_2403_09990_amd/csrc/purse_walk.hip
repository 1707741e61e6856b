// The paper's Step II: the strategic random walk, sampling the rotation
// boundary and the translation boundary separately (Section "The CLOSURE
// Algorithm", Step II; Alg. "d S_R parallel sampler" and, in the appendix
// "Boundary Sampler Algorithms", Alg. "d S_t parallel sampler").
//
// One wavefront per walk.  Per iteration the lanes draw the N_P
// perturbations (up to four per lane), rank them by the distance to the
// boundary min_i (beta_i - ||g_i||_Lambda_i) (eq. partial-s-dist) with N_P*
// rounds of a wavefront argmax (ties to the lower perturbation index), then
// test the N_P* x N_T candidates (up to eight per lane) with in_purse and
// take the one with the largest step scale, then the highest rank, by a
// wavefront minimum of the candidate index m N_P* + k.  The walk's pose is
// wave-uniform (every lane holds the same copy); the keypoints of the
// walk's instance sit in LDS.
#include "purse_fit.hpp"
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

namespace {

constexpr int kWalkWaves = 4;  // walks per workgroup
constexpr int kWalkBlock = 64 * kWalkWaves;

struct WalkKp {
  float m[3];   // model point a_i / Z_i
  float c[3];   // b_i, or (z_i.x, z_i.y, 0); pose regression: t_i
  float w[3];   // 2D-3D: whitening factor of Lambda_i (upper triangle); pose regression:
                // (beta_i^R, beta_i^R + tau, 0)
  float beta;   // beta_i (pose regression: beta_i^t)
  float bt;     // beta_i + tau
  float Ri[9];  // pose regression: the hypothesis' rotation R_i
};

struct WalkInst {
  int kind, n;
  float K[4];
};

// r_i of every keypoint at (R, t): the boundary distance min_i (beta_i - r_i)
// and whether the pose is in S (r_i <= beta_i + tau, depth > z_min).
__device__ __forceinline__ void walk_eval(const WalkKp *kp, const WalkInst &I, const float R[9], const float t[3],
                                          float z_min, float &dist, bool &inside) {
  float d = INFINITY;
  bool ok = true;
  for (int i = 0; i < I.n; ++i) {
    const WalkKp k = kp[i];
    float P[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) P[r] = fmaf(R[3 * r], k.m[0], fmaf(R[3 * r + 1], k.m[1], fmaf(R[3 * r + 2], k.m[2], t[r])));
    float rr;
    if (I.kind == PURSE_KIND_REG) {
      // ||R - R_i||_F and ||t - t_i||: both balls of hypothesis i
      float f = 0.f;
#pragma unroll
      for (int q = 0; q < 9; ++q) f = fmaf(R[q] - k.Ri[q], R[q] - k.Ri[q], f);
      const float rR = sqrtf(f);
      d = fminf(d, k.w[0] - rR);
      ok = ok && (rR <= k.w[1]);
      const float e0 = t[0] - k.c[0], e1 = t[1] - k.c[1], e2 = t[2] - k.c[2];
      rr = sqrtf(fmaf(e0, e0, fmaf(e1, e1, e2 * e2)));
    } else if (I.kind == PURSE_KIND_2D3D) {
      const float iz = 1.f / P[2];
      const float e0 = fmaf(I.K[0], P[0] * iz, I.K[2]) - k.c[0];
      const float e1 = fmaf(I.K[1], P[1] * iz, I.K[3]) - k.c[1];
      const float et0 = fmaf(k.w[0], e0, k.w[1] * e1), et1 = k.w[2] * e1;
      rr = sqrtf(fmaf(et0, et0, et1 * et1));
      ok = ok && (P[2] > z_min);
    } else {
      const float e0 = P[0] - k.c[0], e1 = P[1] - k.c[1], e2 = P[2] - k.c[2];
      rr = sqrtf(fmaf(e0, e0, fmaf(e1, e1, e2 * e2)));
    }
    d = fminf(d, k.beta - rr);
    ok = ok && (rr <= k.bt);
  }
  dist = d;
  inside = ok;
}

// Three 24-bit uniforms of (walk, iteration, perturbation) under key
// (seed, 1 + mode): a direction and a magnitude fraction.
__device__ __forceinline__ void walk_draw(uint64_t seed, int mode, uint64_t walk, uint32_t it, uint32_t j,
                                          float dir[3], float &frac) {
  uint64_t c[4] = {walk, (uint64_t)it, (uint64_t)j, 0ull};
  philox4x64_10(c, seed, 1ull + (uint64_t)mode);
  const float u1 = (float)(c[0] >> 40) * 0x1p-24f;
  const float u2 = (float)(c[1] >> 40) * 0x1p-24f;
  frac = (float)(c[2] >> 40) * 0x1p-24f;
  const float z = 1.f - 2.f * u1;
  const float rho = sqrtf(fmaxf(0.f, 1.f - z * z));
  float sp, cp;
  sincospif(2.f * u2, &sp, &cp);
  dir[0] = rho * cp;
  dir[1] = rho * sp;
  dir[2] = z;
}

__device__ __forceinline__ void left_rotate(const float w[3], const float R[9], float out[9]) {
  float E[9];
  exp_so3(w, E);
  matmul3(E, R, out);
}

// Wavefront argmax of (d, j): larger d, then lower j.
__device__ __forceinline__ void wave_argmax_dj(float &d, int &j) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float d2 = __shfl_xor(d, o, 64);
    const int j2 = __shfl_xor(j, o, 64);
    if (d2 > d || (d2 == d && j2 < j)) {
      d = d2;
      j = j2;
    }
  }
}

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace

// Per instance: the average rotation proj_SO3(sum R0) and translation of its
// starts (the parallel samplers' first lines), in float64.
__global__ void __launch_bounds__(64) k_walk_centre(DevBatch b, const int64_t *__restrict__ start_off,
                                                    int64_t total_starts, const float *__restrict__ starts,
                                                    float *centre) {
  const int j = blockIdx.x, lane = threadIdx.x;
  int64_t s0 = start_off[j], s1 = start_off[j + 1];
  if (s0 < 0 || s1 < s0 || s1 > total_starts) s0 = s1 = 0;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int64_t s = s0 + lane; s < s1; s += 64)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] += (double)starts[12 * s + k];
#pragma unroll
  for (int k = 0; k < 12; ++k)
    for (int o = 32; o >= 1; o >>= 1) acc[k] += __shfl_xor(acc[k], o, 64);
  if (lane == 0) {
    double Rb[9];
    if (s1 > s0) {
      polar_so3<double>(acc, Rb, 12);
    } else {
      for (int k = 0; k < 9; ++k) Rb[k] = (k % 4 == 0) ? 1.0 : 0.0;
    }
    const double inv = s1 > s0 ? 1.0 / (double)(s1 - s0) : 0.0;
    for (int k = 0; k < 9; ++k) centre[12 * j + k] = (float)Rb[k];
    for (int r = 0; r < 3; ++r) centre[12 * j + 9 + r] = (float)(acc[9 + r] * inv);
  }
}

__global__ void __launch_bounds__(kWalkBlock) k_walk(DevBatch b, DevParams p, WalkParams wp,
                                                     const int64_t *__restrict__ start_off, int64_t total_starts,
                                                     const float *__restrict__ starts,
                                                     const float *__restrict__ centre, float *poses, uint8_t *mask,
                                                     int32_t *decisions) {
  __shared__ WalkKp kp_s[kWalkWaves][PURSE_MAX_KP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int mode = blockIdx.y;
  const int64_t n_walks = total_starts * wp.n_walks;
  const int64_t g = (int64_t)blockIdx.x * kWalkWaves + wave;
  if (g >= n_walks) return;  // (whole wavefront)
  const int64_t sg = g / wp.n_walks;
  const int nw = (int)(g % wp.n_walks);
  // instance of start sg: the last j with start_off[j] <= sg
  int lo = 0, hi = b.n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start_off[mid] <= sg)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int j = lo;
  const int64_t out_i = (int64_t)mode * n_walks + g;
  float *out = poses + 12 * out_i;
  float R[9], t[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = starts[12 * sg + k];
#pragma unroll
  for (int r = 0; r < 3; ++r) t[r] = starts[12 * sg + 9 + r];
  WalkInst I;
  I.kind = b.kind[j];
  I.n = b.n_kp[j];
  const int64_t ko = b.kp_off[j];
  const bool valid = (I.kind == PURSE_KIND_3D3D || I.kind == PURSE_KIND_2D3D || I.kind == PURSE_KIND_REG) && I.n >= 1 &&
                     I.n <= PURSE_MAX_KP &&
                     ko >= 0 && b.kp_off[j + 1] - ko == I.n && b.kp_off[j + 1] <= b.total_kp;
  if (!valid) {  // (whole wavefront) the start is returned as it is, not in S
    if (lane < 12) out[lane] = lane < 9 ? R[lane] : t[lane - 9];
    if (lane == 0) mask[out_i] = 0;
    if (decisions)
      for (int it = lane; it < wp.n_iters; it += 64) decisions[out_i * wp.n_iters + it] = -1;
    return;
  }
  const bool is2d = I.kind == PURSE_KIND_2D3D, isreg = I.kind == PURSE_KIND_REG;
  for (int k = 0; k < 4; ++k) I.K[k] = is2d ? b.intrinsics[4 * j + k] : 0.f;
  const float tau = is2d ? p.tau2 : p.tau3;
  WalkKp *kp = kp_s[wave];
  if (lane < I.n) {
    const int64_t q = ko + lane;
    WalkKp k;
    for (int r = 0; r < 3; ++r) {
      k.m[r] = isreg ? 0.f : b.model_pts[3 * q + r];
      k.c[r] = (r < 2 || !is2d) ? b.centres[3 * q + r] : 0.f;
      k.w[r] = 0.f;
    }
    for (int r = 0; r < 9; ++r) k.Ri[r] = 0.f;
    if (is2d) {
      double w[3];
      whiten_factor<double>(b.shapes + 4 * q, w);
      for (int r = 0; r < 3; ++r) k.w[r] = (float)w[r];
    }
    if (isreg) {
      // hypothesis i: rotation from its unit quaternion (shapes), its
      // rotation bound (model_pts x)
      const float *qq = b.shapes + 4 * q;
      const float n = rsqrtf(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
      rot_from_quat(make_float4(qq[0] * n, qq[1] * n, qq[2] * n, qq[3] * n), k.Ri);
      k.w[0] = b.model_pts[3 * q];
      k.w[1] = b.model_pts[3 * q] + tau;
    }
    k.beta = b.bounds[q];
    k.bt = b.bounds[q] + tau;
    kp[lane] = k;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const uint64_t seed = b.seed[j];
  const uint64_t walk = (uint64_t)((sg - start_off[j]) * wp.n_walks + nw);  // instance-local walk index
  // initial velocity: radial direction from the centre of the starts plus a
  // random unit vector
  float vel[3];
  {
    float dir[3], frac;
    walk_draw(seed, mode, walk, 0xFFFFFFFFu, 0u, dir, frac);
    const float *C = centre + 12 * j;
    float u[3];
    if (mode == 0) {
      float Y[9];
      // R0 R_bar^T
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Y[3 * r + c] = R[3 * r] * C[3 * c] + R[3 * r + 1] * C[3 * c + 1] + R[3 * r + 2] * C[3 * c + 2];
      log_so3(Y, u);
    } else {
      for (int r = 0; r < 3; ++r) u[r] = t[r] - C[9 + r];
    }
    const float n2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const float in = n2 > 0.f ? rsqrtf(n2) : 0.f;
    const float mag = mode == 0 ? wp.omega0 : wp.v0;
    for (int r = 0; r < 3; ++r) vel[r] = mag * (u[r] * in + dir[r]);
  }
  const int NP = wp.n_perturb, K = wp.n_keep, NT = wp.n_scales;
  const float pscale = mode == 0 ? wp.t_pert : wp.r_pert;
  for (int it = 0; it < wp.n_iters; ++it) {
    // ---- N_P perturbations, their boundary distances
    float dq[4];
    int jq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = lane + 64 * q;
      jq[q] = jj;
      dq[q] = -INFINITY;
      if (jj < NP) {
        float dir[3], frac;
        walk_draw(seed, mode, walk, (uint32_t)it, (uint32_t)jj, dir, frac);
        const float s = pscale * frac;
        float Rj[9], tj[3];
        if (mode == 0) {
#pragma unroll
          for (int k = 0; k < 9; ++k) Rj[k] = R[k];
#pragma unroll
          for (int r = 0; r < 3; ++r) tj[r] = fmaf(s, dir[r], t[r]);
        } else {
          const float w[3] = {s * dir[0], s * dir[1], s * dir[2]};
          left_rotate(w, R, Rj);
#pragma unroll
          for (int r = 0; r < 3; ++r) tj[r] = t[r];
        }
        bool inside;
        walk_eval(kp, I, Rj, tj, p.z_min, dq[q], inside);
      }
    }
    // ---- the N_P* largest, in rank order
    int keep[kWalkMaxKeep];
    for (int k = 0; k < K; ++k) {
      float bd = -INFINITY;
      int bj = INT32_MAX;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (jq[q] < NP && (dq[q] > bd || (dq[q] == bd && jq[q] < bj))) {
          bd = dq[q];
          bj = jq[q];
        }
      wave_argmax_dj(bd, bj);
      keep[k] = bj;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (jq[q] == bj) jq[q] = INT32_MAX;  // picked
    }
    // ---- candidates (m, k): the largest feasible step, then the best rank
    int best = INT32_MAX;
    const int C = NT * K;
    for (int c = lane; c < C; c += 64) {
      const int m = c / K, k = c % K;
      float dir[3], frac;
      walk_draw(seed, mode, walk, (uint32_t)it, (uint32_t)keep[k], dir, frac);
      const float s = pscale * frac;
      float scale = 1.f;
      for (int q = 0; q < m; ++q) scale *= wp.gamma;
      float Rc[9], tc[3];
      if (mode == 0) {
        const float w[3] = {vel[0] * scale, vel[1] * scale, vel[2] * scale};
        left_rotate(w, R, Rc);
#pragma unroll
        for (int r = 0; r < 3; ++r) tc[r] = fmaf(s, dir[r], t[r]);
      } else {
        const float w[3] = {s * dir[0], s * dir[1], s * dir[2]};
        left_rotate(w, R, Rc);
#pragma unroll
        for (int r = 0; r < 3; ++r) tc[r] = fmaf(vel[r], scale, t[r]);
      }
      float dd;
      bool inside;
      walk_eval(kp, I, Rc, tc, p.z_min, dd, inside);
      if (inside) best = min(best, c);
    }
    best = wave_min_int(best);
    int code = -1;
    if (best != INT32_MAX) {
      // every lane takes the winning candidate (wave-uniform arithmetic)
      const int m = best / K, k = best % K;
      float dir[3], frac;
      walk_draw(seed, mode, walk, (uint32_t)it, (uint32_t)keep[k], dir, frac);
      const float s = pscale * frac;
      float scale = 1.f;
      for (int q = 0; q < m; ++q) scale *= wp.gamma;
      float Rn[9];
      if (mode == 0) {
        const float w[3] = {vel[0] * scale, vel[1] * scale, vel[2] * scale};
        left_rotate(w, R, Rn);
#pragma unroll
        for (int r = 0; r < 3; ++r) t[r] = fmaf(s, dir[r], t[r]);
      } else {
        const float w[3] = {s * dir[0], s * dir[1], s * dir[2]};
        left_rotate(w, R, Rn);
#pragma unroll
        for (int r = 0; r < 3; ++r) t[r] = fmaf(vel[r], scale, t[r]);
      }
#pragma unroll
      for (int k2 = 0; k2 < 9; ++k2) R[k2] = Rn[k2];
      code = k * NT + m;
    }
    if (decisions && lane == 0) decisions[out_i * wp.n_iters + it] = code;
  }
  float dd;
  bool inside;
  walk_eval(kp, I, R, t, p.z_min, dd, inside);
  if (lane < 12) out[lane] = lane < 9 ? R[lane] : t[lane - 9];
  if (lane == 0) mask[out_i] = inside ? PURSE_MASK_FEASIBLE : 0;
}

void launch_walk(const DevBatch &b, const DevParams &p, const WalkParams &wp, const int64_t *start_off,
                 int64_t total_starts, const float *starts, float *centre, float *poses, uint8_t *mask,
                 int32_t *decisions, hipStream_t stream) {
  hipLaunchKernelGGL(k_walk_centre, dim3(b.n_inst), dim3(64), 0, stream, b, start_off, total_starts, starts, centre);
  const int64_t n_walks = total_starts * wp.n_walks;
  if (n_walks == 0) return;
  const dim3 grid((unsigned)((n_walks + kWalkWaves - 1) / kWalkWaves), 2u);
  hipLaunchKernelGGL(k_walk, grid, dim3(kWalkBlock), 0, stream, b, p, wp, start_off, total_starts, starts, centre,
                     poses, mask, decisions);
}

}  // namespace purse
