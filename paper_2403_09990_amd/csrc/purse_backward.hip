// Backward of purse_sample + purse_megb with every discrete decision held as
// taken (argmax trace, feasibility and bisection outcomes, clamp sides).
//
// 1. k_bwd_megb (one workgroup per instance): the rotation iterates are the
//    forward's own float32 ones: every ckpt_every-th is a checkpoint that
//    purse_megb left (or, for a trace it did not produce, that a replay of the
//    descent from the trace writes); the cotangents of (D_hat, d_hat, R*, t*) are swept back through the
//    centre projection, the last-iterate average and the T geodesic steps
//    onto the few samples the trace touches (the active set): the 3x3
//    tangent Jacobians of the steps are formed in float64 in parallel, a
//    chunk of steps at a time, each step's iterate recomputed from its
//    checkpoint, and their products composed by a log-depth scan.
// 2. k_bwd_frame: per input direction, the tangent of the centre fit, pivot
//    and anchor (the fit re-run in float64 dual numbers from its start).
// 3. k_bwd_traj: per (active sample, input direction), the trajectory re-run
//    in float32 dual numbers gives the tangent of the sample's pose, dotted
//    with its cotangent.
// 4. k_bwd_reduce: per direction, the sum over active samples in a fixed
//    order, scattered into the gradient arrays.
#include <mutex>

#include "purse_bwd_check.hpp"
#include "purse_fit.hpp"
#include "purse_geodesic.hpp"
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

namespace {

constexpr int kBwdBlock = 256;
constexpr int kBwdWaves = kBwdBlock / 64;
constexpr int kLdsTrace = 8192;  // descents up to this length are replayed from LDS
constexpr int kTrajGroup = 16;  // lanes per direction in the 2D-3D tangent kernel
static_assert(kMaxActive <= 256, "active-set slots are bytes");

using D = double;

// C = A^T B
__device__ __forceinline__ void matmul_tn(const D A[9], const D B[9], D C[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) C[3 * r + c] = A[r] * B[c] + A[3 + r] * B[3 + c] + A[6 + r] * B[6 + c];
}

// v(X) = vee(X - X^T), so that <X, [w]x> = w . v(X)
__device__ __forceinline__ void vskew(const D X[9], D v[3]) {
  v[0] = X[7] - X[5];
  v[1] = X[2] - X[6];
  v[2] = X[3] - X[1];
}

__device__ __forceinline__ void hat_d(const D w[3], D W[9]) {
  W[0] = 0;
  W[1] = -w[2];
  W[2] = w[1];
  W[3] = w[2];
  W[4] = 0;
  W[5] = -w[0];
  W[6] = -w[1];
  W[7] = w[0];
  W[8] = 0;
}

// One descent step C_i = C Exp(Log(C^T R) / i), over float64 or its dual numbers.
template <typename T>
__device__ __forceinline__ void step_rot_t(const T C[9], const T R[9], int i, T Cn[9]) {
  T Y[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[3 * r + c] = C[r] * R[c] + C[3 + r] * R[3 + c] + C[6 + r] * R[6 + c];
  T w[3], phi[3], E[9];
  log_so3<T>(Y, w);
  const double inv = 1.0 / (double)i;
  phi[0] = w[0] * inv;
  phi[1] = w[1] * inv;
  phi[2] = w[2] * inv;
  exp_so3<T>(phi, E);
  matmul3<T>(C, E, Cn);
}

// Rotation matrix of a (renormalised) float quaternion (w, x, y, z), in float64.
__device__ __forceinline__ void rot_of_quat_d(float4 qf, D R[9]) {
  D w = qf.x, x = qf.y, y = qf.z, z = qf.w;
  const D n = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= n;
  x *= n;
  y *= n;
  z *= n;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

__device__ __forceinline__ void load_R(const float *poses, int64_t g, D R[9]) {
  const float *P = poses + 12 * g;
  for (int k = 0; k < 9; ++k) R[k] = (D)P[k];
}

__device__ __forceinline__ int find_active(const int *act, int n, int s) { return find_sorted(act, n, s); }

}  // namespace

__global__ void __launch_bounds__(kBwdBlock) k_bwd_megb(DevBatch b, DevParams p, const float *__restrict__ poses,
                                                        const uint8_t *__restrict__ mask,
                                                        const int32_t *__restrict__ trace,
                                                        const double *__restrict__ g_radii,
                                                        const float *__restrict__ g_centre,
                                                        const InstRec *__restrict__ inst, MegbRec *megb,
                                                        BwdRec *recs, float4 *ckpt_all, int ck) {
  __shared__ int act[kMaxActive];
  __shared__ int n_act_s, err_s, n_distinct_s;  // err_s: a BwdRec status (kBwdOk while the sweep may run)
  __shared__ double cot[kMaxActive][12];
  __shared__ float pact[kMaxActive][12];       // poses of the active samples
  __shared__ float4 qact[kMaxActive];          // their rotations as quaternions
  __shared__ uint8_t tslot[2 * kLdsTrace];     // trace as active-set slots
  __shared__ double jac[kBwdBlock][2][9];      // J_C, J_R of the steps of one chunk
  __shared__ double jadd[kBwdBlock][3];        // averaged-iterate terms of those steps, then rho terms
  __shared__ double gstep[kBwdBlock][3];       // g at each step of the chunk
  __shared__ int cslot[kBwdBlock];             // active slot of each step of the chunk (rotation)
  __shared__ int tslot_c[kBwdBlock];           // and of its translation winner
  __shared__ double twt[kBwdBlock];            // translation weight of each step of the chunk
  __shared__ double tbar[3];                   // cotangent of t*
  __shared__ double rho[kMaxActive][3];        // tangent cotangents of active rotations
  __shared__ double Sbar_s[9], gvec[3];
  __shared__ double Rstar[9], tstar[3], Ssum[9];
  __shared__ double red_v[kBwdWaves];
  __shared__ int red_i[kBwdWaves];
  __shared__ int s0_s, sD_s, sd_s;
  __shared__ unsigned long long red_h[kBwdWaves];
  __shared__ int stored_s;
  const int j = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int T = p.megb_iters;
  const int avg = p.megb_avg < T ? p.megb_avg : T;
  int64_t off, M64;
  sample_range(b.sample_off, j, b.total_samples, b.max_samples, off, M64);
  const int M = (int)M64;
  BwdRec *rec = recs + j;
  // ---- the prologue's records must belong to this batch and its data (else
  // they would index keypoints of another batch): the instance record's
  // ranges and key, and the fingerprint of the inputs, recomputed here
  if (tid == 0) {
    s0_s = INT32_MAX;
    err_s = inst_record_ok(inst[j], inst_view(b, j)) ? kBwdOk : kBwdStale;
  }
  __syncthreads();
  if (wave == 0 && err_s == kBwdOk) {
    const int n = b.n_kp[j];
    const int64_t ko = b.kp_off[j];
    unsigned long long h = 0ull;
    if (lane < n) {
      const int64_t k = ko + lane;
      uint32_t w[11];
      kp_words(b.kind[j], b.model_pts + 3 * k, b.centres + 3 * k, b.shapes + 4 * k, b.bounds[k], w);
      h = kp_data_term(lane, w);
    }
    for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
    if (lane == 0) {
      const InstRec &I = inst[j];
      h += I.kind == PURSE_KIND_2D3D ? intrinsics_term(I.K) : 0ull;
      if (h != I.data_fp) err_s = kBwdStale;
    }
  }
  __syncthreads();
  if (err_s != kBwdOk) {
    if (tid == 0) {
      rec->n_act = 0;
      rec->n_distinct = 0;
      rec->status = err_s;
    }
    return;
  }
  // ---- first feasible sample: rounds of 8 masks per thread (loads issued
  // together), stopping at the first round that holds one
  for (int r0 = 0; r0 < M; r0 += 8 * kBwdBlock) {
    uint8_t m8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) m8[u] = mask[off + min(r0 + u * kBwdBlock + tid, M - 1)];
    int first = INT32_MAX;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int s = r0 + u * kBwdBlock + tid;
      if (s < M && (m8[u] & PURSE_MASK_FEASIBLE)) first = min(first, s);
    }
    for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
    if (lane == 0 && first != INT32_MAX) atomicMin(&s0_s, first);
    __syncthreads();
    const bool found = s0_s != INT32_MAX;
    __syncthreads();  // every wave has read s0_s before any wave's next round may write it
    if (found) break;
  }
  const int s0 = s0_s;
  if (s0 == INT32_MAX) {
    if (tid == 0) {
      rec->n_act = 0;
      rec->n_distinct = 0;
      rec->status = kBwdEmpty;
    }
    return;
  }
  // ---- active set: the sorted distinct samples of the trace and the first
  // sample, extracted by repeated block minima (the set has tens of members)
  const int32_t *tr = trace + (int64_t)j * T * 2;
  {
    int bad = 0;
    for (int k = tid; k < 2 * T; k += kBwdBlock) {
      int v = tr[k];
      if (v < 0 || v >= M || !(mask[off + v] & PURSE_MASK_FEASIBLE)) bad = 1;
    }
    bad = __syncthreads_or(bad);
    if (bad) {
      if (tid == 0) {
        rec->n_act = 0;
        rec->n_distinct = 0;
        rec->status = kBwdBadTrace;
      }
      return;
    }
  }
  // ---- the rotation checkpoints purse_megb left are used when their
  // signature (steps, winners, the bits of the start's and the winners'
  // rotations) matches this descent (else it is replayed below)
  {
    unsigned long long h = 0ull;
    for (int i = tid; i <= T; i += kBwdBlock) {
      const int id = i == 0 ? s0 : tr[2 * (i - 1)];  // (checked above: samples of the instance)
      uint32_t R[9];
      const float *P = poses + 12 * (off + id);
      for (int k = 0; k < 9; ++k) R[k] = __float_as_uint(P[k]);
      h += step_sig_term(i, id, R);
    }
    for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
    if (lane == 0) red_h[wave] = h;
    __syncthreads();
    if (tid == 0) {
      unsigned long long t = 0ull;
      for (int w = 0; w < kBwdWaves; ++w) t += red_h[w];
      const MegbRec &mr = megb[j];
      stored_s = !(p.flags & PURSE_FLAG_REPLAY_DESCENT) && mr.ck_T == T && mr.ck_every == ck && mr.ck_hash == t;
      if (!stored_s) {
        // the replay below rewrites the checkpoints: they then belong to this trace
        megb[j].ck_hash = t;
        megb[j].ck_T = 0;  // (set to T once written)
        megb[j].ck_every = ck;
      }
      n_act_s = 0;
      n_distinct_s = 0;
    }
  }
  __syncthreads();
  int last = -1;
  while (true) {
    int mn = INT32_MAX;
    for (int k = tid; k <= 2 * T; k += kBwdBlock) {
      int v = k < 2 * T ? tr[k] : s0;
      if (v > last && v < mn) mn = v;
    }
    for (int o = 32; o >= 1; o >>= 1) mn = min(mn, __shfl_xor(mn, o, 64));
    if (lane == 0) red_i[wave] = mn;
    __syncthreads();
    mn = INT32_MAX;
    for (int w = 0; w < kBwdWaves; ++w) mn = min(mn, red_i[w]);
    __syncthreads();
    if (mn == INT32_MAX) break;
    if (tid == 0) {
      ++n_distinct_s;
      if (n_act_s < kMaxActive)
        act[n_act_s++] = mn;
      else
        err_s = kBwdOverflow;
    }
    last = mn;
  }
  __syncthreads();
  // ---- stage the active samples' poses and the trace (as slots) in LDS: the
  // serial sweeps below then read nothing from global memory per step
  // (every active id is a sample of the instance: the trace was checked and
  // s0 was found in range; a trace entry missing from the set would be a
  // bookkeeping error, reported instead of used as a slot)
  const bool lds_trace = T <= kLdsTrace;
  auto stage_active = [&](int n_act_now) {
    int miss = 0;
    if (err_s == kBwdOk) {
      for (int k = tid; k < n_act_now * 12; k += kBwdBlock)
        pact[k / 12][k % 12] = poses[12 * (off + act[k / 12]) + k % 12];
      if (lds_trace)
        for (int k = tid; k < 2 * T; k += kBwdBlock) {
          const int sl = find_active(act, n_act_now, tr[k]);
          miss |= sl < 0;
          tslot[k] = (uint8_t)(sl < 0 ? 0 : sl);
        }
    }
    const bool stop = err_s != kBwdOk;  // (last written before the barrier that ended the previous step)
    miss = __syncthreads_or(miss);
    if (miss && tid == 0) err_s = kBwdBadTrace;
    for (int a = tid; a < n_act_now && !miss && !stop; a += kBwdBlock) qact[a] = quat_from_rot(pact[a]);
    __syncthreads();
  };
  stage_active(n_act_s);
  auto slot_of = [&](int k) {
    if (lds_trace) return (int)tslot[k];
    const int sl = find_active(act, n_act_s, tr[k]);
    return sl < 0 ? 0 : sl;  // (staging checked that every entry has a slot)
  };
  auto load_act = [&](int a, D R[9]) {
    for (int q = 0; q < 9; ++q) R[q] = (D)pact[a][q];
  };
  // ---- the rotation iterates.  The chain repeats the forward's float32
  // quaternion steps, so the backward linearises at the iterates the forward
  // computed; C_0, C_ck, C_2ck, ... are the checkpoints.  With the forward's
  // checkpoints only the last avg iterates are recomputed (from the one at or
  // before step T - avg); otherwise wavefront 0 replays the whole descent
  // (every lane runs the same steps, 1/i and the winners' quaternions from
  // per-lane tables of the next 64 steps) and writes the checkpoints.
  float4 *ckq = ckpt_all + (int64_t)j * ckpt_count(T, ck);
  const bool stored = stored_s != 0;
  if (wave == 0 && err_s == kBwdOk) {
    D S[9];
    for (int k = 0; k < 9; ++k) S[k] = 0;
    if (stored) {
      const int q0 = (T - avg) / ck;
      float4 C = ckq[q0];
      for (int i = q0 * ck + 1; i <= T; ++i) {
        C = geodesic_step(C, qact[slot_of(2 * (i - 1))], i, 0);
        if (i > T - avg) {
          D Cm[9];
          rot_of_quat_d(C, Cm);
          for (int k = 0; k < 9; ++k) S[k] += Cm[k];
        }
      }
    } else {
      float4 C = qact[max(find_active(act, n_act_s, s0), 0)];  // (s0 is in the set)
      int ib = 1, kc = 0, q = 0;
      float inv_tab = 1.f / (float)(ib + lane);
      float4 B_tab = qact[slot_of(2 * min(ib - 1 + lane, T - 1))];
      for (int i = 1; i <= T; ++i) {
        if (i - ib == 64) {
          ib = i;
          inv_tab = 1.f / (float)(ib + lane);
          B_tab = qact[slot_of(2 * min(ib - 1 + lane, T - 1))];
        }
        const int l = i - ib;
        const float inv = readlane_f(inv_tab, l);
        const float4 B = make_float4(readlane_f(B_tab.x, l), readlane_f(B_tab.y, l), readlane_f(B_tab.z, l),
                                     readlane_f(B_tab.w, l));
        if (kc == 0) {  // (i - 1) % ck == 0
          if (lane == 0) ckq[q] = C;
          ++q;
          kc = ck;
        }
        --kc;
        C = geodesic_step_inv(C, B, inv, i, 0);
        if (i > T - avg) {
          D Cm[9];
          rot_of_quat_d(C, Cm);
          for (int k = 0; k < 9; ++k) S[k] += Cm[k];
        }
      }
    }
    if (lane == 0) {
      D Rs[9];
      polar_so3<D>(S, Rs, 12);
      for (int k = 0; k < 9; ++k) {
        Rstar[k] = Rs[k];
        Ssum[k] = S[k];
      }
      if (!stored) megb[j].ck_T = T;
    }
  }
  // ---- t* = (1/avg) sum_{i > T - avg} c_i, where c_i (c_i = c_{i-1} + (t_{s_i}
  // - c_{i-1}) / i, c_1 = t_{s_1}) is the mean of the first i winners: winner
  // k carries (1/avg) sum_{i >= max(k, T - avg + 1)} 1/i.  All threads, in
  // float64, summed in a fixed order.
  if (err_s == kBwdOk) {
    D hs = 0;
    for (int k = T - avg + 1; k <= T; ++k) hs += 1.0 / (D)k;
    D ta[3] = {0.0, 0.0, 0.0};
    for (int k = 1 + tid; k <= T; k += kBwdBlock) {
      D w = hs;
      if (k > T - avg) {
        w = 0;
        for (int m = k; m <= T; ++m) w += 1.0 / (D)m;
      }
      const float *P = pact[slot_of(2 * (k - 1) + 1)];
      for (int r = 0; r < 3; ++r) ta[r] += w * (D)P[9 + r];
    }
    for (int o = 1; o < 64; o <<= 1)
      for (int r = 0; r < 3; ++r) ta[r] += __shfl_xor(ta[r], o, 64);
    if (lane == 0)
      for (int r = 0; r < 3; ++r) gstep[wave][r] = ta[r];
  }
  __syncthreads();
  if (tid == 0 && err_s == kBwdOk) {
    for (int r = 0; r < 3; ++r) {
      D t = 0;
      for (int w = 0; w < kBwdWaves; ++w) t += gstep[w][r];
      tstar[r] = t / avg;
    }
    // a non-finite centre has no radius samples
    bool fin = true;
    for (int k = 0; k < 9; ++k) fin = fin && isfinite(Rstar[k]);
    for (int k = 0; k < 3; ++k) fin = fin && isfinite(tstar[k]);
    if (!fin) err_s = kBwdNonFinite;
  }
  __syncthreads();
  // ---- samples realising the radii about (R*, t*)
  D br = -1, bt = -1;
  int ir = INT32_MAX, it = INT32_MAX;
  {
    // 4 samples per thread and round, their loads issued together
    constexpr int U = 4;
    D Rs[9], ts[3];
    for (int k = 0; k < 9; ++k) Rs[k] = Rstar[k];
    for (int k = 0; k < 3; ++k) ts[k] = tstar[k];
    for (int r0 = 0; r0 < M; r0 += U * kBwdBlock) {
      float4 q[U][3];
      uint8_t m4[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int s = min(r0 + u * kBwdBlock + tid, M - 1);
        const float4 *P = reinterpret_cast<const float4 *>(poses + 12 * (off + s));
        q[u][0] = P[0];
        q[u][1] = P[1];
        q[u][2] = P[2];
        m4[u] = mask[off + s];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int s = r0 + u * kBwdBlock + tid;
        if (s >= M || !(m4[u] & PURSE_MASK_FEASIBLE)) continue;
        const float P[12] = {q[u][0].x, q[u][0].y, q[u][0].z, q[u][0].w, q[u][1].x, q[u][1].y,
                             q[u][1].z, q[u][1].w, q[u][2].x, q[u][2].y, q[u][2].z, q[u][2].w};
        D fr = 0, ft = 0;
        for (int k = 0; k < 9; ++k) {
          D d = Rs[k] - (D)P[k];
          fr += d * d;
        }
        for (int k = 0; k < 3; ++k) {
          D d = ts[k] - (D)P[9 + k];
          ft += d * d;
        }
        // increasing s per thread: a strictly larger value replaces the best
        radius_take(fr, s, br, ir);
        radius_take(ft, s, bt, it);
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) radius_merge(__shfl_xor(br, o, 64), __shfl_xor(ir, o, 64), br, ir);
  if (lane == 0) {
    red_v[wave] = br;
    red_i[wave] = ir;
  }
  __syncthreads();
  if (tid == 0) {
    D v = red_v[0];
    int ii = red_i[0];
    for (int w = 1; w < kBwdWaves; ++w) radius_merge(red_v[w], red_i[w], v, ii);
    sD_s = ii;
  }
  __syncthreads();
  for (int o = 32; o >= 1; o >>= 1) radius_merge(__shfl_xor(bt, o, 64), __shfl_xor(it, o, 64), bt, it);
  if (lane == 0) {
    red_v[wave] = bt;
    red_i[wave] = it;
  }
  __syncthreads();
  if (tid == 0) {
    D v = red_v[0];
    int ii = red_i[0];
    for (int w = 1; w < kBwdWaves; ++w) radius_merge(red_v[w], red_i[w], v, ii);
    sd_s = ii;
    // insert the radius samples into the sorted active set; an id that is no
    // sample of the instance (the search's sentinel, left when no distance
    // compared) ends the backward of this instance instead of indexing poses
    if (err_s == kBwdOk) {
      int32_t st = radius_sample_status(sD_s, M);
      if (st == kBwdOk) st = radius_sample_status(sd_s, M);
      if (st == kBwdOk) st = active_insert(act, n_act_s, kMaxActive, sD_s, M);
      if (st == kBwdOk) st = active_insert(act, n_act_s, kMaxActive, sd_s, M);
      if (st != kBwdOk) err_s = st;
    }
  }
  for (int k = tid; k < kMaxActive * 12; k += kBwdBlock) cot[k / 12][k % 12] = 0.0;
  __syncthreads();
  const int n_act = n_act_s;
  // a radius sample outside the trace shifts the active set: stage the poses
  // and the trace slots again for the new positions
  stage_active(n_act);
  // ---- reverse sweeps
  // Rotation chain.  Thread 0 turns the cotangents of R* and the rotation
  // radius into S_bar = dL/dS (S = sum of the last iterates).  Then the T
  // steps are swept backwards in chunks of kBwdBlock: every thread takes one
  // step i of the chunk, recomputes C_{i-1} from its checkpoint and, in dual
  // numbers, the 3x3 Jacobians of C_i = C_{i-1} Exp(Log(C_{i-1}^T R) / i) in
  // right-trivialised tangents, J_C (w.r.t. C_{i-1} Exp(d)) and J_R (w.r.t.
  // R Exp(e)); thread 0 then runs the chunk's recurrence
  //   g_i += vskew(C_i^T S_bar) (i among the averaged iterates),
  //   rho_{s_i} += J_R^T g_i,  g_{i-1} = J_C^T g_i,
  // so the serial part is 3x3 products only.  g_0 belongs to the first
  // sample (C_0 = R_{s0}); a sample's tangent cotangent rho becomes the
  // ambient cotangent R [rho]x / 2 of its rotation.
  if (tid == 0 && err_s == kBwdOk) {
    // cotangent of R*: (g_w . left tangent) and the rotation radius
    D G[9], W[9];
    // the left so(3) cotangent at R*; a cotangent of R*'s entries G gives
    // vskew(G R*^T) (the pairing <G, [w]x R*> = w . vskew(G R*^T))
    const bool mat = (p.flags & PURSE_FLAG_MATRIX_COTANGENT) != 0;
    const float *gc = g_centre + (mat ? 12 : 6) * j;
    D gw[3] = {gc[0], gc[1], gc[2]};
    if (mat) {
      D X[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          X[3 * r + c] = (D)gc[3 * r] * Rstar[3 * c] + (D)gc[3 * r + 1] * Rstar[3 * c + 1] + (D)gc[3 * r + 2] * Rstar[3 * c + 2];
      vskew(X, gw);
    }
    hat_d(gw, W);
    matmul3<D>(W, Rstar, G);
    for (int k = 0; k < 9; ++k) G[k] *= 0.5;
    D RD[9];
    load_R(poses, off + sD_s, RD);
    D f2 = 0;
    for (int k = 0; k < 9; ++k) f2 += (Rstar[k] - RD[k]) * (Rstar[k] - RD[k]);
    const D gD = g_radii[2 * j];
    if (f2 > 0 && gD != 0) {
      D f = sqrt(f2);
      D x = f / (2.0 * sqrt(2.0));
      D kD = gD / (sqrt(2.0) * sqrt(fmax(1e-30, 1.0 - x * x)) * f);
      const int pD = max(find_active(act, n_act, sD_s), 0);  // (inserted above)
      for (int k = 0; k < 9; ++k) {
        D v = kD * (Rstar[k] - RD[k]);
        G[k] += v;
        cot[pD][k] -= v;
      }
    }
    // through R* = polar(S): S_bar = R* [b]x, b = (tr H I - H)^-1 v(R*^T G), H = sym(R*^T S)
    D RtG[9], H[9], vv[3];
    matmul_tn(Rstar, G, RtG);
    vskew(RtG, vv);
    D RtS[9];
    matmul_tn(Rstar, Ssum, RtS);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) H[3 * r + c] = 0.5 * (RtS[3 * r + c] + RtS[3 * c + r]);
    D trH = H[0] + H[4] + H[8];
    D h00 = trH - H[0], h11 = trH - H[4], h22 = trH - H[8], h01 = -H[1], h02 = -H[2], h12 = -H[5];
    D a00 = h11 * h22 - h12 * h12, a01 = h02 * h12 - h01 * h22, a02 = h01 * h12 - h02 * h11;
    D a11 = h00 * h22 - h02 * h02, a12 = h01 * h02 - h00 * h12, a22 = h00 * h11 - h01 * h01;
    D det = h00 * a00 + h01 * a01 + h02 * a02;
    D bb[3] = {(a00 * vv[0] + a01 * vv[1] + a02 * vv[2]) / det, (a01 * vv[0] + a11 * vv[1] + a12 * vv[2]) / det,
               (a02 * vv[0] + a12 * vv[1] + a22 * vv[2]) / det};
    D Bh[9], Sbar[9];
    hat_d(bb, Bh);
    matmul3<D>(Rstar, Bh, Sbar);
    for (int k = 0; k < 9; ++k) Sbar_s[k] = Sbar[k];
    for (int k = 0; k < 3; ++k) gvec[k] = 0.0;
  }
  for (int k = tid; k < kMaxActive * 3; k += kBwdBlock) rho[k / 3][k % 3] = 0.0;
  __syncthreads();
  // Translation chain: c_i = c_{i-1} + (t_{s_i} - c_{i-1}) / i is linear, so
  // its reverse is a scalar recurrence per coordinate, swept by thread 64 over
  // each chunk while thread 0 sweeps the rotation chain.
  D tb[3] = {0, 0, 0};
  if (tid == 64 && err_s == kBwdOk) {
    const bool mat = (p.flags & PURSE_FLAG_MATRIX_COTANGENT) != 0;
    const float *gc = g_centre + (mat ? 12 : 6) * j + (mat ? 9 : 3);
    tb[0] = gc[0];
    tb[1] = gc[1];
    tb[2] = gc[2];
    const D gd = g_radii[2 * j + 1];
    const float *Pd = poses + 12 * (off + sd_s);
    D dv[3] = {tstar[0] - Pd[9], tstar[1] - Pd[10], tstar[2] - Pd[11]};
    D dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    if (dn > 0 && gd != 0) {
      const int pd = max(find_active(act, n_act, sd_s), 0);  // (inserted above)
      for (int r = 0; r < 3; ++r) {
        tb[r] += gd * dv[r] / dn;
        cot[pd][9 + r] -= gd * dv[r] / dn;
      }
    }
    for (int r = 0; r < 3; ++r) tbar[r] = tb[r];
  }
  // Translation chain in closed form: t* = (1/avg) sum_{k > T - avg} c_{k+1}
  // with c_{k+1} the mean of the first k winners, so step i's winner gets
  // tbar (1/avg) sum_{k >= max(i, T - avg + 1)} 1/k; hsum = that sum for the
  // steps before the last avg.
  D hsum = 0;
  for (int k = T - avg + 1; k <= T; ++k) hsum += 1.0 / (D)k;
  __syncthreads();
  if (err_s == kBwdOk) {
    for (int i_hi = T; i_hi >= 1; i_hi -= kBwdBlock) {
      const int i_lo = max(1, i_hi - kBwdBlock + 1);
      const int i = i_lo + tid;
      if (i <= i_hi) {
        // C_{i-1}: the forward's float32 steps from the checkpoint C_{q ck}, q = (i - 1) / ck
        const int q = (i - 1) / ck;
        float4 Cf = ckq[q];
        for (int m = q * ck + 1; m <= i - 1; ++m) Cf = geodesic_step(Cf, qact[slot_of(2 * (m - 1))], m, 0);
        D C[9];
        rot_of_quat_d(Cf, C);
        D R[9];
        load_act(slot_of(2 * (i - 1)), R);
        D Ci[9];
        step_rot_t<D>(C, R, i, Ci);
        // ambient term of the averaged iterates
        D a[3] = {0.0, 0.0, 0.0};
        if (i > T - avg) {
          D Sb[9], X[9];
          for (int k = 0; k < 9; ++k) Sb[k] = Sbar_s[k];
          matmul_tn(Ci, Sb, X);
          vskew(X, a);
        }
        // Jacobian columns from right perturbations of C_{i-1} and of R
        for (int which = 0; which < 2; ++which)
          for (int c = 0; c < 3; ++c) {
            Dual<D> Cd[9], Rd[9], Cnd[9];
            for (int k = 0; k < 9; ++k) {
              Cd[k] = Dual<D>(C[k], 0.0);
              Rd[k] = Dual<D>(R[k], 0.0);
            }
            // X [e_c]x: column c2 of X [e]x is X (e x e_c2)
            Dual<D> *X = which == 0 ? Cd : Rd;
            const D *Xv = which == 0 ? C : R;
            for (int r = 0; r < 3; ++r) {
              const D x0 = Xv[3 * r], x1 = Xv[3 * r + 1], x2 = Xv[3 * r + 2];
              // [e_c]x columns: e_c x e_0, e_c x e_1, e_c x e_2
              D d0 = 0, d1 = 0, d2 = 0;
              if (c == 0) { d1 = x2; d2 = -x1; }
              if (c == 1) { d0 = -x2; d2 = x0; }
              if (c == 2) { d0 = x1; d1 = -x0; }
              X[3 * r].d = d0;
              X[3 * r + 1].d = d1;
              X[3 * r + 2].d = d2;
            }
            step_rot_t<Dual<D>>(Cd, Rd, i, Cnd);
            D dC[9], Y[9], v[3];
            for (int k = 0; k < 9; ++k) dC[k] = Cnd[k].d;
            matmul_tn(Ci, dC, Y);
            vskew(Y, v);
            for (int r = 0; r < 3; ++r) jac[tid][which][3 * r + c] = 0.5 * v[r];
          }
        for (int k = 0; k < 3; ++k) jadd[tid][k] = a[k];
      }
      __syncthreads();
      {
        // g through the chunk's steps: with g_i the cotangent entering step i
        // (from above), step i leaves J_C^T (g_i + a_i), an affine map F_i of
        // g_i, and keeps g_i + a_i.  The g_i of all steps come from suffix
        // compositions S_t = F_t o ... o F_top of the chunk's maps, formed by
        // a log-depth scan (each level composes with the map d steps below),
        // the maps exchanged through the J_C slots and gstep.
        const int n = i_hi - i_lo + 1;
        D M[9], bv[3], at[3];
        if (tid < n) {
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[3 * r + c] = jac[tid][0][3 * c + r];  // J_C^T
          for (int k = 0; k < 3; ++k) at[k] = jadd[tid][k];
          for (int r = 0; r < 3; ++r) bv[r] = M[3 * r] * at[0] + M[3 * r + 1] * at[1] + M[3 * r + 2] * at[2];
        }
        for (int d = 1; d < n; d <<= 1) {
          __syncthreads();
          if (tid < n) {
            for (int k = 0; k < 9; ++k) jac[tid][0][k] = M[k];
            for (int k = 0; k < 3; ++k) gstep[tid][k] = bv[k];
          }
          __syncthreads();
          if (tid + d < n) {
            // S_t o S_{t+d}: S_{t+d} (the steps above) first
            D M2[9], b2[3], Mn[9];
            for (int k = 0; k < 9; ++k) M2[k] = jac[tid + d][0][k];
            for (int k = 0; k < 3; ++k) b2[k] = gstep[tid + d][k];
            for (int r = 0; r < 3; ++r) {
              for (int c = 0; c < 3; ++c) Mn[3 * r + c] = M[3 * r] * M2[c] + M[3 * r + 1] * M2[3 + c] + M[3 * r + 2] * M2[6 + c];
              bv[r] += M[3 * r] * b2[0] + M[3 * r + 1] * b2[1] + M[3 * r + 2] * b2[2];
            }
            for (int k = 0; k < 9; ++k) M[k] = Mn[k];
          }
        }
        __syncthreads();
        if (tid < n) {
          for (int k = 0; k < 9; ++k) jac[tid][0][k] = M[k];
          for (int k = 0; k < 3; ++k) gstep[tid][k] = bv[k];
        }
        __syncthreads();
        const D g0[3] = {gvec[0], gvec[1], gvec[2]};
        D gb[3] = {g0[0], g0[1], g0[2]}, gout[3];
        if (tid + 1 < n) {
          const D *Mu = jac[tid + 1][0];
          const D *bu = gstep[tid + 1];
          for (int r = 0; r < 3; ++r) gb[r] = Mu[3 * r] * g0[0] + Mu[3 * r + 1] * g0[1] + Mu[3 * r + 2] * g0[2] + bu[r];
        }
        if (tid == 0)
          for (int r = 0; r < 3; ++r) gout[r] = M[3 * r] * g0[0] + M[3 * r + 1] * g0[1] + M[3 * r + 2] * g0[2] + bv[r];
        __syncthreads();
        if (tid < n)
          for (int k = 0; k < 3; ++k) gstep[tid][k] = gb[k] + at[k];
        if (tid == 0)
          for (int k = 0; k < 3; ++k) gvec[k] = gout[k];
      }
      __syncthreads();
      // rho_{s_i} += J_R^T g_i: each step's term in parallel, then summed per
      // active sample in step order (deterministic; every term read by every
      // summing thread, selected by its slot)
      if (i <= i_hi) {
        const D *JR = jac[tid][1];
        for (int c = 0; c < 3; ++c) jadd[tid][c] = JR[c] * gstep[tid][0] + JR[3 + c] * gstep[tid][1] + JR[6 + c] * gstep[tid][2];
        cslot[tid] = slot_of(2 * (i - 1));
        D h = hsum;
        if (i > T - avg) {
          h = 0;
          for (int k = i; k <= T; ++k) h += 1.0 / (D)k;
        }
        twt[tid] = h / avg;
        tslot_c[tid] = slot_of(2 * (i - 1) + 1);
      } else {
        cslot[tid] = -1;
        tslot_c[tid] = -1;
      }
      __syncthreads();
      // per active sample (one wavefront each): the rotation terms into rho,
      // the translation weights into the cotangent; lane l sums steps 4l ..
      // 4l + 3, then a butterfly of fixed shape (the same sums every run)
      static_assert(kBwdBlock == 4 * 64, "four steps of the chunk per lane");
      for (int a = wave; a < n_act; a += kBwdWaves) {
        D v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 3; u >= 0; --u) {
          const int t = 4 * lane + u;
          const bool m = cslot[t] == a;
          v[0] += m ? jadd[t][0] : 0.0;
          v[1] += m ? jadd[t][1] : 0.0;
          v[2] += m ? jadd[t][2] : 0.0;
          v[3] += tslot_c[t] == a ? twt[t] : 0.0;
        }
        for (int o = 1; o < 64; o <<= 1)
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] += __shfl_xor(v[k], o, 64);
        if (lane == 0) {
          rho[a][0] += v[0];
          rho[a][1] += v[1];
          rho[a][2] += v[2];
          for (int r = 0; r < 3; ++r) cot[a][9 + r] += tbar[r] * v[3];
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int p0 = max(find_active(act, n_act, s0), 0);  // (s0 is in the set)
      for (int k = 0; k < 3; ++k) rho[p0][k] += gvec[k];
    }
    __syncthreads();
    // rho -> ambient cotangent R [rho]x / 2
    for (int a = tid; a < n_act; a += kBwdBlock) {
      D R[9], Wr[9], X[9];
      load_act(a, R);
      hat_d(rho[a], Wr);
      matmul3<D>(R, Wr, X);
      for (int k = 0; k < 9; ++k) cot[a][k] += 0.5 * X[k];
    }
  }
  __syncthreads();
  if (tid == 0) {
    rec->n_act = err_s != kBwdOk ? 0 : n_act;
    rec->n_distinct = n_distinct_s;
    rec->status = err_s;
    rec->s0 = s0;
    rec->sD = sD_s;
    rec->sd = sd_s;
  }
  const int n_out = err_s != kBwdOk ? 0 : n_act;
  for (int k = tid; k < n_out * 12; k += kBwdBlock) rec->cot[k / 12][k % 12] = cot[k / 12][k % 12];
  for (int k = tid; k < n_out; k += kBwdBlock) rec->active[k] = act[k];
}

// ---------------------------------------------------------------------------
// input directions: 3D-3D d = 4 i + c (b_i.x, b_i.y, b_i.z, beta_i);
// 2D-3D d = 6 i + c (z_i.x, z_i.y, Lambda_00, Lambda_01 = Lambda_10, Lambda_11, beta_i)
__device__ __forceinline__ int dirs_per_kp(int kind) { return kind == PURSE_KIND_2D3D ? 6 : 4; }

// Tangent of keypoint i_d's constraint data along direction component c.
__device__ void kp_tangent(const InstRec &I, const KpRec &k, const float *shapes_i, float beta_i, float kappa,
                           int c, KpT<Dual<float>> &o) {
  for (int r = 0; r < 3; ++r) {
    o.m[r] = k.m[r];
    o.c[r] = Dual<float>(k.c[r], 0.f);
    o.w[r] = Dual<float>(k.w[r], 0.f);
  }
  o.kb = Dual<float>(k.kb, 0.f);
  o.kb2 = Dual<float>(k.kb2, 0.f);
  o.bt = Dual<float>(k.bt, 0.f);
  const bool is2d = I.kind == PURSE_KIND_2D3D;
  const int cb = is2d ? 5 : 3;
  if (c == cb) {
    o.kb.d = kappa;
    o.kb2.d = 2.f * k.kb * kappa;
    o.bt.d = 1.f;
  } else if (!is2d || c < 2) {
    o.c[c].d = 1.f;
  } else {
    double w[3];
    whiten_factor<double>(shapes_i, w);
    double dw0 = 0, dw1 = 0, dw2 = 0;
    if (c == 2) {
      dw0 = 0.5 / w[0];
      dw1 = -w[1] * dw0 / w[0];
      dw2 = -w[1] * dw1 / w[2];
    } else if (c == 3) {
      dw1 = 1.0 / w[0];
      dw2 = -w[1] * dw1 / w[2];
    } else {
      dw2 = 0.5 / w[2];
    }
    o.w[0].d = (float)dw0;
    o.w[1].d = (float)dw1;
    o.w[2].d = (float)dw2;
  }
}

struct KpDual {
  static constexpr bool kPrefetch = false;
  const KpRec *__restrict__ kp;
  int i_d;
  KpT<Dual<float>> tk;
  __device__ __forceinline__ KpT<Dual<float>> operator()(int i) const {
    if (i == i_d) return tk;
    const KpRec k = kp[i];
    KpT<Dual<float>> o;
    for (int r = 0; r < 3; ++r) {
      o.m[r] = k.m[r];
      o.c[r] = Dual<float>(k.c[r], 0.f);
      o.w[r] = Dual<float>(k.w[r], 0.f);
    }
    o.kb = Dual<float>(k.kb, 0.f);
    o.kb2 = Dual<float>(k.kb2, 0.f);
    o.bt = Dual<float>(k.bt, 0.f);
    return o;
  }
};

// 2D-3D observations with the tangent of one keypoint.
struct ObsDual {
  const float *z;
  const float *shapes;
  int i_d, c;
  __device__ void operator()(int i, Dual<double> zz[2], Dual<double> w[3]) const {
    double wv[3];
    whiten_factor<double>(shapes + 4 * i, wv);
    zz[0] = Dual<double>((double)z[3 * i], 0.0);
    zz[1] = Dual<double>((double)z[3 * i + 1], 0.0);
    for (int r = 0; r < 3; ++r) w[r] = Dual<double>(wv[r], 0.0);
    if (i != i_d) return;
    if (c < 2) {
      zz[c].d = 1.0;
    } else if (c == 2) {
      w[0].d = 0.5 / wv[0];
      w[1].d = -wv[1] * w[0].d / wv[0];
      w[2].d = -wv[1] * w[1].d / wv[2];
    } else if (c == 3) {
      w[1].d = 1.0 / wv[0];
      w[2].d = -wv[1] * w[1].d / wv[2];
    } else if (c == 4) {
      w[2].d = 0.5 / wv[2];
    }
  }
};

// Tangent of the centre, pivot and anchor along one input direction.
// (It reads nothing k_bwd_megb writes, so the two run concurrently.)
__global__ void __launch_bounds__(kMaxDirs) k_bwd_frame(DevBatch b, DevParams p, const InstRec *__restrict__ inst,
                                                       const KpRec *__restrict__ kprec, float *tan_all,
                                                       int max_dirs) {
  const int j = blockIdx.x;
  const int d = threadIdx.x;
  const InstRec I = inst[j];
  // (whole workgroup) a record of another batch is not used: k_bwd_megb
  // reports it and no tangent is read for that instance
  if (!inst_record_ok(I, inst_view(b, j)) || (I.status & 0xFF) != PURSE_INST_OK) return;
  const bool is2d = I.kind == PURSE_KIND_2D3D;
  const int dpk = dirs_per_kp(I.kind);
  const int n = I.n_kp;
  const float *a = b.model_pts + 3 * I.kp_off;
  const float *cz = b.centres + 3 * I.kp_off;
  const float *L = b.shapes + 4 * I.kp_off;
  // 2D-3D: the forward's choice between the two starts, made once for all
  // directions: wavefront 0 fits from the DLT start, wavefront 1 from the
  // weak-perspective start (whitening factors cached), as the prologue does
  __shared__ double w_s[3 * PURSE_MAX_KP];
  __shared__ double st_R[2][9], st_t[2][3], st_cost[2];
  __shared__ int st_ok[2];
  if (is2d) {
    for (int i = d; i < n; i += blockDim.x) whiten_factor<double>(L + 4 * i, w_s + 3 * i);
    __syncthreads();
    if (d == 0 || d == 64) {
      const int f = d >> 6;
      const ObsCached obs{cz, w_s};
      double R[9], t[3], R0[9], t0[3];
      bool ok = f == 0 ? dlt_2d(a, cz, n, I.K, R, t) : affine_2d(a, cz, n, I.K, R, t);
      for (int k = 0; k < 9; ++k) R0[k] = R[k];
      for (int k = 0; k < 3; ++k) t0[k] = t[k];
      if (ok) ok = gn_centre_2d<double>(a, obs, n, I.K, p.centre_gn, (double)p.z_min, R, t);
      st_ok[f] = ok;
      for (int k = 0; k < 9; ++k) st_R[f][k] = R0[k];  // the start, not the fit
      for (int k = 0; k < 3; ++k) st_t[f][k] = t0[k];
      st_cost[f] = ok ? cost_2d_obs(a, obs, n, I.K, R, t) : 0.0;
    }
    __syncthreads();
  }
  if (d >= n * dpk) return;
  const int i_d = d / dpk, c = d % dpk;
  Dual<double> Rd[9], td[3];
  if (!is2d) {
    // Arun's fit with b_{i_d} perturbed
    double ab[3] = {0, 0, 0};
    Dual<double> bb[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < 3; ++r) {
        ab[r] += a[3 * i + r];
        bb[r] += Dual<double>((double)cz[3 * i + r], (i == i_d && r == c) ? 1.0 : 0.0);
      }
    for (int r = 0; r < 3; ++r) {
      ab[r] /= n;
      bb[r] = bb[r] / (double)n;
    }
    Dual<double> H[9];
    for (int k = 0; k < 9; ++k) H[k] = Dual<double>(0.0, 0.0);
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < 3; ++r) {
        Dual<double> br = Dual<double>((double)cz[3 * i + r], (i == i_d && r == c) ? 1.0 : 0.0) - bb[r];
        for (int q = 0; q < 3; ++q) H[3 * r + q] += br * ((double)a[3 * i + q] - ab[q]);
      }
    polar_so3<Dual<double>>(H, Rd, 12);
    for (int r = 0; r < 3; ++r) td[r] = bb[r] - (Rd[3 * r] * ab[0] + Rd[3 * r + 1] * ab[1] + Rd[3 * r + 2] * ab[2]);
  } else {
    // from the start whose fit the forward kept (lower cost; ties: the DLT one)
    const bool ok1 = st_ok[0] != 0, ok2 = st_ok[1] != 0;
    const int f = (ok2 && (!ok1 || st_cost[1] < st_cost[0])) ? 1 : 0;
    for (int k = 0; k < 9; ++k) Rd[k] = Dual<double>(st_R[f][k], 0.0);
    for (int k = 0; k < 3; ++k) td[k] = Dual<double>(st_t[f][k], 0.0);
    const ObsDual od{cz, L, i_d, c};
    gn_centre_2d<Dual<double>>(a, od, n, I.K, p.centre_gn, (double)p.z_min, Rd, td);
  }
  FrameT<Dual<float>> F;
  for (int k = 0; k < 9; ++k) F.Rc[k] = Dual<float>(I.Rc[k], (float)Rd[k].d);
  for (int r = 0; r < 3; ++r) F.tc[r] = Dual<float>(I.tc[r], (float)td[r].d);
  for (int r = 0; r < 3; ++r) {
    double od = Rd[3 * r].d * I.abar[0] + Rd[3 * r + 1].d * I.abar[1] + Rd[3 * r + 2].d * I.abar[2] + td[r].d;
    F.oc[r] = Dual<float>(I.oc[r], (float)od);
  }
  for (int k = 0; k < 9; ++k) F.Ra[k] = F.Rc[k];
  for (int r = 0; r < 3; ++r) F.ta[r] = F.tc[r];
  if ((I.status & PURSE_INST_ANCHOR_ITERATED) && I.has_anchor) {
    KpDual kpl;
    kpl.kp = kprec + I.kp_off;
    kpl.i_d = i_d;
    kp_tangent(I, kprec[I.kp_off + i_d], L + 4 * i_d, b.bounds[I.kp_off + i_d], p.kappa, c, kpl.tk);
    PoseT<Dual<float>> x;
    for (int k = 0; k < 9; ++k) x.R[k] = F.Rc[k];
    for (int r = 0; r < 3; ++r) x.t[r] = F.tc[r];
    int nfb = 0;
    if (is2d)
      run_trajectory<PURSE_KIND_2D3D>(I, F, kpl, x, p, false, nfb);
    else
      run_trajectory<PURSE_KIND_3D3D>(I, F, kpl, x, p, false, nfb);
    for (int k = 0; k < 9; ++k) F.Ra[k] = Dual<float>(I.Ra[k], x.R[k].d);
    for (int r = 0; r < 3; ++r) F.ta[r] = Dual<float>(I.ta[r], x.t[r].d);
  }
  float *tan = tan_all + ((int64_t)j * max_dirs + d) * 27;
  for (int k = 0; k < 9; ++k) tan[k] = F.Rc[k].d;
  for (int r = 0; r < 3; ++r) tan[9 + r] = F.tc[r].d;
  for (int r = 0; r < 3; ++r) tan[12 + r] = F.oc[r].d;
  for (int k = 0; k < 9; ++k) tan[15 + k] = F.Ra[k].d;
  for (int r = 0; r < 3; ++r) tan[24 + r] = F.ta[r].d;
}

// Work items of the tangent kernels: instance j contributes n_act_j x zb_j
// items (zb_j workgroups of 64 lanes cover its directions, `lanes` lanes per
// direction), listed by an exclusive prefix sum over the instances of the
// kind, so a fixed grid walks exactly the items the active sets need
// (instead of a grid sized for full active sets, which dispatches mostly
// empty workgroups).
__device__ __forceinline__ int item_blocks(int n_kp, int kind, int lanes) {
  return (n_kp * dirs_per_kp(kind) * lanes + 63) / 64;
}

__global__ void __launch_bounds__(1024) k_bwd_items(DevBatch b, const InstRec *__restrict__ inst,
                                                    const BwdRec *recs, int kind, int lanes,
                                                    int64_t *__restrict__ item_off) {
  __shared__ int64_t part[1024];
  const int n = b.n_inst, tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int j0 = tid * per, j1 = min(n, j0 + per);
  auto items_of = [&](int j) -> int64_t {
    const BwdRec &r = recs[j];
    const InstRec I = inst[j];
    if (r.status != kBwdOk || I.kind != kind || (I.status & 0xFF) != PURSE_INST_OK || !inst_record_ok(I, inst_view(b, j)))
      return 0;
    return (int64_t)min(max(r.n_act, 0), kMaxActive) * item_blocks(I.n_kp, kind, lanes);
  };
  int64_t acc = 0;
  for (int j = j0; j < j1; ++j) acc += items_of(j);
  part[tid] = acc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t run = tid ? part[tid - 1] : 0;
  for (int j = j0; j < j1; ++j) {
    item_off[j] = run;
    run += items_of(j);
  }
  if (tid == 1023) item_off[n] = part[1023];
}

// Item -> (instance, active slot, block of directions).
__device__ __forceinline__ void item_at(const int64_t *__restrict__ item_off, int n, int64_t it, const InstRec *inst,
                                        int kind, int lanes, int &j, int &a, int &z) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {  // the last instance whose range starts at or before it
    const int mid = (lo + hi + 1) >> 1;
    if (item_off[mid] <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  j = lo;
  const int zb = item_blocks(inst[j].n_kp, kind, lanes);
  const int64_t local = it - item_off[j];
  a = (int)(local / zb);
  z = (int)(local % zb);
}

constexpr int kItemGrid = 8192;  // workgroups of the tangent kernels (each walks items kItemGrid apart)

// Tangent of active sample a's pose along 64 directions, dotted with its
// cotangent; one work item per workgroup iteration.
template <int KIND>
__global__ void __launch_bounds__(64) k_bwd_traj(DevBatch b, DevParams p, const InstRec *__restrict__ inst,
                                                 const KpRec *__restrict__ kprec, const BwdRec *recs,
                                                 const int64_t *__restrict__ item_off,
                                                 const float *__restrict__ tan_all, float *contrib, int max_dirs) {
  const int64_t total = item_off[b.n_inst];
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    int j, a, z;
    item_at(item_off, b.n_inst, it, inst, KIND, 1, j, a, z);
    const int d = z * 64 + threadIdx.x;
    const BwdRec *rec = recs + j;
    // (listed only when k_bwd_megb of this call found the instance record
    // to match the batch and its data, and the active set within capacity)
    const InstRec I = inst[j];
    const int dpk = dirs_per_kp(KIND);
    if (d >= I.n_kp * dpk) continue;
    const int i_d = d / dpk, c = d % dpk;
    const float *tan = tan_all + ((int64_t)j * max_dirs + d) * 27;
    FrameT<Dual<float>> F;
    for (int k = 0; k < 9; ++k) {
      F.Rc[k] = Dual<float>(I.Rc[k], tan[k]);
      F.Ra[k] = Dual<float>(I.Ra[k], tan[15 + k]);
    }
    for (int r = 0; r < 3; ++r) {
      F.tc[r] = Dual<float>(I.tc[r], tan[9 + r]);
      F.oc[r] = Dual<float>(I.oc[r], tan[12 + r]);
      F.ta[r] = Dual<float>(I.ta[r], tan[24 + r]);
    }
    KpDual kpl;
    kpl.kp = kprec + I.kp_off;
    kpl.i_d = i_d;
    kp_tangent(I, kprec[I.kp_off + i_d], b.shapes + 4 * (I.kp_off + i_d), b.bounds[I.kp_off + i_d], p.kappa, c,
               kpl.tk);
    const int s = rec->active[a];
    PoseT<Dual<float>> x = initial_pose<Dual<float>>(F, I.seed, (uint64_t)s, p);
    int nfb = 0;
    const uint8_t m = run_trajectory<KIND>(I, F, kpl, x, p, true, nfb);
    double acc = 0.0;
    if (m & PURSE_MASK_FEASIBLE) {
      for (int k = 0; k < 9; ++k) acc += rec->cot[a][k] * (double)x.R[k].d;
      for (int r = 0; r < 3; ++r) acc += rec->cot[a][9 + r] * (double)x.t[r].d;
    }
    contrib[((int64_t)j * kMaxActive + a) * max_dirs + d] = (float)acc;
  }
}

// ---------------------------------------------------------------------------
// 2D-3D tangents with G lanes per (active sample, direction): lane q of a
// group takes the keypoints i = q, q + G, ...; the normal equations and the
// depth and feasibility tests are combined across the group by DPP lane
// permutations (butterfly sums: every lane of the group ends with the same
// value, addition being commutative), so each lane carries 1/G of the
// keypoint work and a small batch of active samples fills G times more
// wavefronts.  The arithmetic per keypoint is that of gn_pass2d.
template <int G>
__device__ __forceinline__ float group_sum(float x) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "lane groups within a row of 16");
  x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
  if (G >= 4) x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  if (G >= 8) x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x141, 0xF, 0xF, false));  // half mirror
  if (G >= 16) x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x140, 0xF, 0xF, false));  // row mirror
  return x;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int G>
__device__ __forceinline__ double group_sum(double x) {
  static_assert(G == 2 || G == 4 || G == 8 || G == 16, "lane groups within a row of 16");
  x += dpp_f64<0xB1>(x);
  if (G >= 4) x += dpp_f64<0x4E>(x);
  if (G >= 8) x += dpp_f64<0x141>(x);
  if (G >= 16) x += dpp_f64<0x140>(x);
  return x;
}

template <int G>
__device__ __forceinline__ Dual<float> group_sum(Dual<float> x) {
  return Dual<float>(group_sum<G>(x.v), group_sum<G>(x.d));
}

template <int G>
__device__ __forceinline__ bool group_and(bool b) {
  int v = b ? 1 : 0;
  v &= __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
  if (G >= 4) v &= __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
  if (G >= 8) v &= __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
  if (G >= 16) v &= __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);
  return v != 0;
}

using DF = Dual<float>;

template <bool FIRST, int G>
__device__ __forceinline__ bool gn_pass2d_group(const KpDual &kpl, int n, int q, const float K[4], const DF oc[3],
                                                float z_min, float band, const PoseT<DF> &xk, PoseT<DF> &x) {
  DF A[21], g[6];
  for (int k = 0; k < 21; ++k) A[k] = DF(0.f);
  for (int k = 0; k < 6; ++k) g[k] = DF(0.f);
  bool ok = true;
  for (int i = q; i < n; i += G) {
    const auto k = kpl(i);
    DF P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    ok = ok && (P[2] > z_min);
    DF rt0, rt1;
    if (FIRST) {
      DF e0 = u - k.c[0], e1 = v - k.c[1];
      DF et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
      DF r2 = et0 * et0 + et1 * et1;
      DF sc = (r2 <= k.kb2 * band) ? DF(1.f) : k.kb * drsqrt(r2);
      rt0 = (sc - 1.f) * et0;
      rt1 = (sc - 1.f) * et1;
    } else {
      DF Pk[3], izk, uk, vk;
      project2d(xk.R, xk.t, k, K, Pk, izk, uk, vk);
      DF e0 = uk - k.c[0], e1 = vk - k.c[1];
      DF et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
      DF r2 = et0 * et0 + et1 * et1;
      DF sc = (r2 <= k.kb2 * band) ? DF(1.f) : k.kb * drsqrt(r2);
      DF r0 = k.c[0] + sc * e0 - u, r1 = k.c[1] + sc * e1 - v;
      rt0 = k.w[0] * r0 + k.w[1] * r1;
      rt1 = k.w[2] * r1;
    }
    DF pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
    gn_accumulate<DF>(P, pt, iz, DF(K[0]), DF(K[1]), k.w, rt0, rt1, A, g);
  }
  for (int k = 0; k < 21; ++k) A[k] = group_sum<G>(A[k]);
  for (int k = 0; k < 6; ++k) g[k] = group_sum<G>(g[k]);
  ok = group_and<G>(ok);
  DF d[6];
  ok = ok && chol6_solve<DF>(A, g, d);
  if (!ok) return false;
  apply_update<DF>(d, oc, x.R, x.t);
  return true;
}

template <int G>
__device__ __forceinline__ bool feasible2d_group(const KpDual &kpl, int n, int q, const float K[4],
                                                 const PoseT<DF> &x, float z_min) {
  bool ok = true;
  for (int i = q; i < n; i += G) {
    const auto k = kpl(i);
    DF P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    DF e0 = u - k.c[0], e1 = v - k.c[1];
    DF et0 = k.w[0] * e0 + k.w[1] * e1, et1 = k.w[2] * e1;
    const float rr = sqrtf(value_of(et0 * et0 + et1 * et1));
    ok = ok && (value_of(P[2]) > z_min) && (rr <= value_of(k.bt));
  }
  return group_and<G>(ok);
}

// run_trajectory (2D-3D) on a lane group: iterations, feasibility test,
// bisection pull-in towards the anchor.
template <int G, typename FR>
__device__ __forceinline__ uint8_t run_trajectory_group(const InstRec &I, const FR &F, const KpDual &kpl, int q,
                                                        PoseT<DF> &x, const DevParams &p) {
  const float band = ClampBand<DF>::v;
  const DF oc[3] = {DF(F.oc[0]), DF(F.oc[1]), DF(F.oc[2])};
  bool ok = true;
  for (int it = 0; it < p.n_iters && ok; ++it) {
    const PoseT<DF> xk = x;
    ok = gn_pass2d_group<true, G>(kpl, I.n_kp, q, I.K, oc, p.z_min, band, xk, x);
    for (int gs = 1; gs < p.n_gn && ok; ++gs) ok = gn_pass2d_group<false, G>(kpl, I.n_kp, q, I.K, oc, p.z_min, band, xk, x);
  }
  reorthonormalise(x.R);
  if (!ok) return PURSE_MASK_FAILED;
  if (feasible2d_group<G>(kpl, I.n_kp, q, I.K, x, p.z_min)) return PURSE_MASK_FEASIBLE;
  if (!I.has_anchor) return 0;
  DF Ra[9], ta[3], RtR[9], RaT[9], w[3];
  for (int k = 0; k < 9; ++k) Ra[k] = F.Ra[k];
  for (int r = 0; r < 3; ++r) ta[r] = F.ta[r];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) RaT[3 * r + c] = Ra[3 * c + r];
  matmul3(RaT, x.R, RtR);
  log_so3(RtR, w);
  float lo = 0.f, hi = 1.f;
  for (int b = 0; b < p.n_bis; ++b) {
    const float mid = 0.5f * (lo + hi);
    DF wm[3] = {mid * w[0], mid * w[1], mid * w[2]}, E[9];
    PoseT<DF> m;
    exp_so3(wm, E);
    matmul3(Ra, E, m.R);
    for (int r = 0; r < 3; ++r) m.t[r] = ta[r] + mid * (x.t[r] - ta[r]);
    if (feasible2d_group<G>(kpl, I.n_kp, q, I.K, m, p.z_min))
      lo = mid;
    else
      hi = mid;
  }
  if (lo == 0.f) {
    for (int k = 0; k < 9; ++k) x.R[k] = Ra[k];
    for (int r = 0; r < 3; ++r) x.t[r] = ta[r];
  } else {
    DF wl[3] = {lo * w[0], lo * w[1], lo * w[2]}, E[9];
    exp_so3(wl, E);
    DF Rn[9];
    matmul3(Ra, E, Rn);
    for (int k = 0; k < 9; ++k) x.R[k] = Rn[k];
    for (int r = 0; r < 3; ++r) x.t[r] = ta[r] + lo * (x.t[r] - ta[r]);
  }
  return PURSE_MASK_FEASIBLE | PURSE_MASK_PULLED_IN;
}

// k_bwd_traj for 2D-3D instances with G lanes per direction: work item
// (j, a, z) covers active sample a and directions z * 64 / G ... of instance j.
template <int G>
__global__ void __launch_bounds__(64) k_bwd_traj2d_group(DevBatch b, DevParams p, const InstRec *__restrict__ inst,
                                                         const KpRec *__restrict__ kprec, const BwdRec *recs,
                                                         const int64_t *__restrict__ item_off,
                                                         const float *__restrict__ tan_all, float *contrib,
                                                         int max_dirs) {
  const int64_t total = item_off[b.n_inst];
  const int q = threadIdx.x % G;
  for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
    int j, a, z;
    item_at(item_off, b.n_inst, it, inst, PURSE_KIND_2D3D, G, j, a, z);
    const int d = z * (64 / G) + threadIdx.x / G;
    const BwdRec *rec = recs + j;
    // (see k_bwd_traj)
    const InstRec I = inst[j];
    const int dpk = dirs_per_kp(PURSE_KIND_2D3D);
    if (d >= I.n_kp * dpk) continue;  // (whole lane groups)
    const int i_d = d / dpk, c = d % dpk;
    const float *tan = tan_all + ((int64_t)j * max_dirs + d) * 27;
    FrameT<DF> F;
    for (int k = 0; k < 9; ++k) {
      F.Rc[k] = DF(I.Rc[k], tan[k]);
      F.Ra[k] = DF(I.Ra[k], tan[15 + k]);
    }
    for (int r = 0; r < 3; ++r) {
      F.tc[r] = DF(I.tc[r], tan[9 + r]);
      F.oc[r] = DF(I.oc[r], tan[12 + r]);
      F.ta[r] = DF(I.ta[r], tan[24 + r]);
    }
    KpDual kpl;
    kpl.kp = kprec + I.kp_off;
    kpl.i_d = i_d;
    kp_tangent(I, kprec[I.kp_off + i_d], b.shapes + 4 * (I.kp_off + i_d), b.bounds[I.kp_off + i_d], p.kappa, c,
               kpl.tk);
    const int s = rec->active[a];
    PoseT<DF> x = initial_pose<DF>(F, I.seed, (uint64_t)s, p);
    const uint8_t m = run_trajectory_group<G>(I, F, kpl, q, x, p);
    if (q == 0) {
      double acc = 0.0;
      if (m & PURSE_MASK_FEASIBLE) {
        for (int k = 0; k < 9; ++k) acc += rec->cot[a][k] * (double)x.R[k].d;
        for (int r = 0; r < 3; ++r) acc += rec->cot[a][9 + r] * (double)x.t[r].d;
      }
      contrib[((int64_t)j * kMaxActive + a) * max_dirs + d] = (float)acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Reverse-mode tangent pass of 2D-3D trajectories.  The forward-mode kernels
// above re-run an active sample's trajectory once per input direction (6N
// re-runs); the trajectory's derivative is a linear map from the frame and
// keypoint data to the end pose, so one reverse sweep per active sample gives
// the cotangent of all of them, and every direction's contribution is then a
// dot product with that direction's tangent of the frame and of its keypoint.
// The sweep differentiates the same computation as the forward-mode kernels:
// the same clamp band, the same frozen decisions (clamp sets, the feasibility
// and depth tests, the bisection's outcome), float32 throughout.
//
// Layout: kRevGroup lanes per active sample (lane q takes keypoints q, q + 16,
// ...), four samples per wavefront.  A first pass recomputes the trajectory
// and keeps every Gauss-Newton pass's input pose in LDS (the tape); the
// reverse pass then walks the passes backwards, recomputing each pass's
// normal equations from its input pose.  Per pass (x' = Exp(dw) x about the
// pivot, d = A^-1 g):
//   d_bar from the update's adjoint; g_bar = A^-1 d_bar (the same factor);
//   per keypoint and Jacobian row j_r with residual rt_r:
//     rt_bar_r = g_bar . j_r,  j_bar_r = g_bar (rt_r - d . j_r) - d (g_bar . j_r),
//   then back through the rows (pt x d_r, d_r), the whitened projection
//   Jacobian, the residual (the clamp scale s = kappa beta / r when clamped,
//   the second pass's targets from the iteration's first pose) and the
//   projection, into the pose and the keypoint's data; the pivot's
//   cotangent comes whole from each update (rev_pivot_adjoint).
constexpr int kRevGroup = 16;
constexpr int kRevPerLane = (PURSE_MAX_KP + kRevGroup - 1) / kRevGroup;
constexpr int kRevSamples = 64 / kRevGroup;  // active samples per wavefront
constexpr size_t kRevLds = 65536;              // LDS of a reverse-sweep workgroup at most

// LDS of a reverse-sweep workgroup: per sample, a float32 pose per pass (the
// tape) and a byte of clamp bits per lane and iteration.
__host__ __device__ constexpr size_t rev_lds(int passes, int iters) {
  return sizeof(float) * 12 * kRevSamples * (size_t)(passes > 0 ? passes : 1) +
         (size_t)kRevSamples * kRevGroup * (size_t)(iters > 0 ? iters : 1);
}

template <typename T>
struct RevPoseT {
  T R[9], t[3];
};
using RevPose = RevPoseT<float>;

template <typename T>
__device__ __forceinline__ void rev_round(const RevPoseT<T> &x, RevPose &y) {
#pragma unroll
  for (int m = 0; m < 9; ++m) y.R[m] = (float)x.R[m];
#pragma unroll
  for (int m = 0; m < 3; ++m) y.t[m] = (float)x.t[m];
}

// Group-summed normal equations of one pass at x (targets from xk for the
// later passes), as gn_pass2d_group computes them; false on a depth below
// z_min.  Projection decisions: bit rr of cl is lane q's keypoint
// q + kRevGroup rr; taken from cl when use_cl, else decided here and
// recorded in cl.
template <bool FIRST, typename T>
__device__ __forceinline__ bool rev_normal_eqs(const KpRec *__restrict__ kp, int n, int q, const float K[4],
                                               const T oc[3], float z_min, float band, const RevPoseT<T> &xk,
                                               const RevPoseT<T> &x, T A[21], T g[6], uint32_t &cl, bool use_cl) {
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = T(0);
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = T(0);
  bool ok = true;
  if (!use_cl) cl = 0u;
  for (int i = q, rr = 0; i < n; i += kRevGroup, ++rr) {
    const KpRec k = kp[i];
    const T w[3] = {T(k.w[0]), T(k.w[1]), T(k.w[2])};
    T P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    ok = ok && (P[2] > T(z_min));
    T rt0, rt1;
    if (FIRST) {
      const T e0 = u - T(k.c[0]), e1 = v - T(k.c[1]);
      const T et0 = w[0] * e0 + w[1] * e1, et1 = w[2] * e1;
      const T r2 = et0 * et0 + et1 * et1;
      if (!use_cl && !(r2 <= T(k.kb2) * T(band))) cl |= 1u << rr;
      const T s = ((cl >> rr) & 1u) ? T(k.kb) * drsqrt(r2) : T(1);
      rt0 = (s - T(1)) * et0;
      rt1 = (s - T(1)) * et1;
    } else {
      T Pk[3], izk, uk, vk;
      project2d(xk.R, xk.t, k, K, Pk, izk, uk, vk);
      const T e0 = uk - T(k.c[0]), e1 = vk - T(k.c[1]);
      const T et0 = w[0] * e0 + w[1] * e1, et1 = w[2] * e1;
      const T r2 = et0 * et0 + et1 * et1;
      if (!use_cl && !(r2 <= T(k.kb2) * T(band))) cl |= 1u << rr;
      const T s = ((cl >> rr) & 1u) ? T(k.kb) * drsqrt(r2) : T(1);
      const T r0 = T(k.c[0]) + s * e0 - u, r1 = T(k.c[1]) + s * e1 - v;
      rt0 = w[0] * r0 + w[1] * r1;
      rt1 = w[2] * r1;
    }
    const T pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
    gn_accumulate<T>(P, pt, iz, T(K[0]), T(K[1]), w, rt0, rt1, A, g);
  }
#pragma unroll
  for (int k = 0; k < 21; ++k) A[k] = group_sum<kRevGroup>(A[k]);
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = group_sum<kRevGroup>(g[k]);
  return group_and<kRevGroup>(ok);
}

// <E_bar, dExp(w)/dw_k> for k = 0, 1, 2 (the literal exp_so3 differentiated
// by dual numbers, as the forward-mode kernels do).
__device__ __forceinline__ void rev_exp_adjoint(const float w[3], const float Eb[9], float wb[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Dual<float> wd[3] = {Dual<float>(w[0], k == 0 ? 1.f : 0.f), Dual<float>(w[1], k == 1 ? 1.f : 0.f),
                         Dual<float>(w[2], k == 2 ? 1.f : 0.f)};
    Dual<float> E[9];
    exp_so3(wd, E);
    float acc = 0.f;
#pragma unroll
    for (int m = 0; m < 9; ++m) acc += Eb[m] * E[m].d;
    wb[k] = acc;
  }
}

// Cotangent of the pivot o from one Gauss-Newton update, given the cotangent
// t_bar of the updated translation.  In the coordinates (dw, dv + o x dw) the
// linearised fit does not depend on o (a point moves by dw x P + dv - dw x o),
// so at a fixed input pose and fixed targets the update moves the
// translation by (I - E + [dw]x) o, E = Exp(dw); the pivot's cotangent is
// that matrix transposed applied to t_bar: -(1 - A) dw x t_bar
// - B dw x (dw x t_bar), A = sin th / th, B = (1 - cos th) / th^2 (series
// below th^2 = 0.1).  Formed directly, it is second order in the step:
// summing the first-order terms of the update's and of the keypoint rows'
// dependences on o, which cancel, loses it to float32 rounding.
__device__ __forceinline__ void rev_pivot_adjoint(const float dw[3], const float tb[3], float ob[3]) {
  const float th2 = dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2];
  float oma, bb;
  if (th2 < 0.1f) {
    oma = th2 * (1.f / 6.f - th2 * (1.f / 120.f - th2 * (1.f / 5040.f - th2 * (1.f / 362880.f))));
    bb = 0.5f - th2 * (1.f / 24.f - th2 * (1.f / 720.f - th2 * (1.f / 40320.f)));
  } else {
    const float th = sqrtf(th2);
    oma = 1.f - sinf(th) / th;
    bb = (1.f - cosf(th)) / th2;
  }
  float wt[3], wwt[3];
  cross3(dw, tb, wt);
  cross3(dw, wt, wwt);
#pragma unroll
  for (int r = 0; r < 3; ++r) ob[r] -= oma * wt[r] + bb * wwt[r];
}

// Adjoint of the pose update x' = (E R, E (t - o) + o + dv), E = Exp(dw):
// from x_bar' to the cotangents of the input pose (uniform part), of o and
// of the step d = (dw, dv).
__device__ __forceinline__ void rev_update_adjoint(const float d[6], const float o[3], const RevPose &x,
                                                   const RevPose &xb_out, RevPose &xb_in, float ob[3],
                                                   float db[6]) {
  float E[9];
  exp_so3(d, E);
  float Eb[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // R_bar_in = E^T R_bar', t_bar_in = E^T t_bar'
      xb_in.R[3 * r + c] = E[r] * xb_out.R[c] + E[3 + r] * xb_out.R[3 + c] + E[6 + r] * xb_out.R[6 + c];
      // E_bar = R_bar' R^T + t_bar' (t - o)^T
      Eb[3 * r + c] = xb_out.R[3 * r] * x.R[3 * c] + xb_out.R[3 * r + 1] * x.R[3 * c + 1] +
                      xb_out.R[3 * r + 2] * x.R[3 * c + 2] + xb_out.t[r] * (x.t[c] - o[c]);
    }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    xb_in.t[r] = E[r] * xb_out.t[0] + E[3 + r] * xb_out.t[1] + E[6 + r] * xb_out.t[2];
    db[3 + r] = xb_out.t[r];
  }
  rev_pivot_adjoint(d, xb_out.t, ob);
  rev_exp_adjoint(d, Eb, db);
}

// Per-keypoint adjoint of one pass: adds this lane's part of the input
// pose's cotangent (xb), of the iteration's first pose (xkb, later passes)
// and of its keypoints' data (kb: c0, c1, w0, w1, w2, kappa beta).  (The
// pivot's cotangent is taken whole from the update, rev_pivot_adjoint.)
template <bool FIRST>
__device__ __forceinline__ void rev_keypoints(const KpRec *__restrict__ kp, int n, int q, const float K[4],
                                              const float oc[3], uint32_t clbits, const RevPose &xk,
                                              const RevPose &x, const float d[6], const float gb[6],
                                              RevPose &xb, RevPose &xkb, float kb[kRevPerLane][6]) {
#pragma unroll
  for (int rr = 0; rr < kRevPerLane; ++rr) {
    const int i = q + kRevGroup * rr;
    if (i >= n) break;
    const KpRec k = kp[i];
    const float w0 = k.w[0], w1 = k.w[1], w2 = k.w[2];
    float P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    // residual (and what its adjoint needs)
    float rt0, rt1, e0, e1, et0, et1, r2 = 0.f, s = 1.f;
    bool cl = false;
    float Pk[3] = {0.f, 0.f, 0.f}, izk = 0.f;
    if (FIRST) {
      e0 = u - k.c[0];
      e1 = v - k.c[1];
      et0 = w0 * e0 + w1 * e1;
      et1 = w2 * e1;
      r2 = et0 * et0 + et1 * et1;
      cl = (clbits >> rr) & 1u;
      s = cl ? k.kb * drsqrt(r2) : 1.f;
      rt0 = (s - 1.f) * et0;
      rt1 = (s - 1.f) * et1;
    } else {
      float uk, vk;
      project2d(xk.R, xk.t, k, K, Pk, izk, uk, vk);
      e0 = uk - k.c[0];
      e1 = vk - k.c[1];
      et0 = w0 * e0 + w1 * e1;
      et1 = w2 * e1;
      r2 = et0 * et0 + et1 * et1;
      cl = (clbits >> rr) & 1u;
      s = cl ? k.kb * drsqrt(r2) : 1.f;
      const float r0 = k.c[0] + s * e0 - u, r1 = k.c[1] + s * e1 - v;
      rt0 = w0 * r0 + w1 * r1;
      rt1 = w2 * r1;
      // (r0, r1 are needed below: keep them in e-form)
      et0 = r0;  // reuse: r0
      et1 = r1;  // reuse: r1
    }
    const float pt[3] = {P[0] - oc[0], P[1] - oc[1], P[2] - oc[2]};
    const float a = K[0] * iz, cc = K[1] * iz, nx = P[0] * iz, ny = P[1] * iz;
    const float d0[3] = {w0 * a, w1 * cc, -(w0 * a * nx + w1 * cc * ny)};
    const float d1[3] = {0.f, w2 * cc, -w2 * cc * ny};
    float j0[6], j1[6];
    cross3(pt, d0, j0);
    j0[3] = d0[0];
    j0[4] = d0[1];
    j0[5] = d0[2];
    j1[0] = pt[1] * d1[2] - pt[2] * d1[1];
    j1[1] = -pt[0] * d1[2];
    j1[2] = pt[0] * d1[1];
    j1[3] = 0.f;
    j1[4] = d1[1];
    j1[5] = d1[2];
    float al0 = 0.f, al1 = 0.f, be0 = 0.f, be1 = 0.f;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      al0 += d[m] * j0[m];
      al1 += d[m] * j1[m];
      be0 += gb[m] * j0[m];
      be1 += gb[m] * j1[m];
    }
    float jb0[6], jb1[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      jb0[m] = gb[m] * (rt0 - al0) - d[m] * be0;
      jb1[m] = gb[m] * (rt1 - al1) - d[m] * be1;
    }
    // rows (pt x d_r, d_r): d_bar_r = z + y x pt, pt_bar += d_r x y
    float D0[3], D1[3], ptb[3], tmp[3];
    cross3(jb0, pt, tmp);
    D0[0] = jb0[3] + tmp[0];
    D0[1] = jb0[4] + tmp[1];
    D0[2] = jb0[5] + tmp[2];
    cross3(d0, jb0, ptb);
    cross3(jb1, pt, tmp);
    D1[1] = jb1[4] + tmp[1];
    D1[2] = jb1[5] + tmp[2];
    cross3(d1, jb1, tmp);
    ptb[0] += tmp[0];
    ptb[1] += tmp[1];
    ptb[2] += tmp[2];
    // back through d0, d1
    float wb0 = D0[0] * a - D0[2] * a * nx;
    float wb1 = D0[1] * cc - D0[2] * cc * ny;
    float wb2 = D1[1] * cc - D1[2] * cc * ny;
    const float ab = D0[0] * w0 - D0[2] * w0 * nx;
    const float ccb = D0[1] * w1 - D0[2] * w1 * ny + D1[1] * w2 - D1[2] * w2 * ny;
    const float nxb = -D0[2] * w0 * a;
    const float nyb = -D0[2] * w1 * cc - D1[2] * w2 * cc;
    float izb = ab * K[0] + ccb * K[1] + nxb * P[0] + nyb * P[1];
    float Pb[3] = {nxb * iz, nyb * iz, 0.f};
    // residual
    float ub = 0.f, vb = 0.f, cb0 = 0.f, cb1 = 0.f, kbb = 0.f;
    if (FIRST) {
      float etb0 = (s - 1.f) * be0, etb1 = (s - 1.f) * be1;
      if (cl) {
        const float sb = be0 * et0 + be1 * et1;
        kbb += sb * drsqrt(r2);
        const float r2b = -0.5f * sb * s / r2;
        etb0 += 2.f * r2b * et0;
        etb1 += 2.f * r2b * et1;
      }
      wb0 += etb0 * e0;
      wb1 += etb0 * e1;
      wb2 += etb1 * e1;
      const float eb0 = etb0 * w0, eb1 = etb0 * w1 + etb1 * w2;
      ub += eb0;
      vb += eb1;
      cb0 -= eb0;
      cb1 -= eb1;
    } else {
      const float r0 = et0, r1 = et1;
      wb0 += be0 * r0;
      wb1 += be0 * r1;
      wb2 += be1 * r1;
      const float rb0 = be0 * w0, rb1 = be0 * w1 + be1 * w2;
      cb0 += rb0;
      cb1 += rb1;
      ub -= rb0;
      vb -= rb1;
      float ekb0 = s * rb0, ekb1 = s * rb1;
      if (cl) {
        const float skb = rb0 * e0 + rb1 * e1;
        kbb += skb * drsqrt(r2);
        const float r2b = -0.5f * skb * s / r2;
        const float etk0 = w0 * e0 + w1 * e1, etk1 = w2 * e1;
        const float etkb0 = 2.f * r2b * etk0, etkb1 = 2.f * r2b * etk1;
        wb0 += etkb0 * e0;
        wb1 += etkb0 * e1;
        wb2 += etkb1 * e1;
        ekb0 += etkb0 * w0;
        ekb1 += etkb0 * w1 + etkb1 * w2;
      }
      cb0 -= ekb0;
      cb1 -= ekb1;
      // projection at the iteration's first pose
      const float izkb = ekb0 * K[0] * Pk[0] + ekb1 * K[1] * Pk[1];
      const float Pkb[3] = {ekb0 * K[0] * izk, ekb1 * K[1] * izk, -izkb * izk * izk};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        xkb.R[3 * r] += Pkb[r] * k.m[0];
        xkb.R[3 * r + 1] += Pkb[r] * k.m[1];
        xkb.R[3 * r + 2] += Pkb[r] * k.m[2];
        xkb.t[r] += Pkb[r];
      }
    }
    // projection at x, pt = P - o, iz = 1 / P.z, P = R m + t
    Pb[0] += ub * K[0] * iz;
    Pb[1] += vb * K[1] * iz;
    izb += ub * K[0] * P[0] + vb * K[1] * P[1];
#pragma unroll
    for (int r = 0; r < 3; ++r) Pb[r] += ptb[r];
    Pb[2] += -izb * iz * iz;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      xb.R[3 * r] += Pb[r] * k.m[0];
      xb.R[3 * r + 1] += Pb[r] * k.m[1];
      xb.R[3 * r + 2] += Pb[r] * k.m[2];
      xb.t[r] += Pb[r];
    }
    kb[rr][0] += cb0;
    kb[rr][1] += cb1;
    kb[rr][2] += wb0;
    kb[rr][3] += wb1;
    kb[rr][4] += wb2;
    kb[rr][5] += kbb;
  }
}

// One pass of the reverse sweep: the normal equations at x recomputed, the
// update's and the solve's adjoints, the keypoints' adjoints; xb holds the
// cotangent of the pass's output on entry and of its input on return.
template <bool FIRST>
__device__ __forceinline__ void rev_pass(const KpRec *__restrict__ kp, int n, int q, const float K[4],
                                         const float oc[3], float z_min, uint32_t clbits, const RevPose &xk,
                                         const RevPose &x, RevPose &xb, RevPose &xkb, float ob_u[3],
                                         float kb[kRevPerLane][6]) {
  float A[21], g[6], L[21], dinv[6], d[6];
  rev_normal_eqs<FIRST, float>(kp, n, q, K, oc, z_min, 1.f, xk, x, A, g, clbits, true);
  chol6_factor<float>(A, L, dinv);
  chol6_subst<float>(L, dinv, g, d);
  RevPose xin;
  float db[6];
  rev_update_adjoint(d, oc, x, xb, xin, ob_u, db);
  float gb[6];
  chol6_subst<float>(L, dinv, db, gb);
  RevPose part;
#pragma unroll
  for (int m = 0; m < 9; ++m) part.R[m] = 0.f;
#pragma unroll
  for (int m = 0; m < 3; ++m) part.t[m] = 0.f;
  rev_keypoints<FIRST>(kp, n, q, K, oc, clbits, xk, x, d, gb, part, xkb, kb);
  if (FIRST) {
    // the pass's input is the iteration's first pose: the later passes' parts join here
#pragma unroll
    for (int m = 0; m < 9; ++m) part.R[m] += xkb.R[m];
#pragma unroll
    for (int m = 0; m < 3; ++m) part.t[m] += xkb.t[m];
  }
#pragma unroll
  for (int m = 0; m < 9; ++m) xb.R[m] = xin.R[m] + group_sum<kRevGroup>(part.R[m]);
#pragma unroll
  for (int m = 0; m < 3; ++m) xb.t[m] = xin.t[m] + group_sum<kRevGroup>(part.t[m]);
}

// Adjoint of R_r = R (3 I - R^T R) / 2.
__device__ __forceinline__ void rev_reorthonormalise(const float R[9], float Rb[9]) {
  float S[9], F[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) F[m] = Rb[m];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S[3 * r + c] = -(R[r] * R[c] + R[3 + r] * R[3 + c] + R[6 + r] * R[6 + c]);
  S[0] += 3.f;
  S[4] += 3.f;
  S[8] += 3.f;
  // R_bar = (F S - R F^T R - R R^T F) / 2
  float FS[9], RFt[9], RFtR[9], RRt[9], RRtF[9];
  matmul3(F, S, FS);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      RFt[3 * r + c] = R[3 * r] * F[3 * c] + R[3 * r + 1] * F[3 * c + 1] + R[3 * r + 2] * F[3 * c + 2];
      RRt[3 * r + c] = R[3 * r] * R[3 * c] + R[3 * r + 1] * R[3 * c + 1] + R[3 * r + 2] * R[3 * c + 2];
    }
  matmul3(RFt, R, RFtR);
  matmul3(RRt, F, RRtF);
#pragma unroll
  for (int m = 0; m < 9; ++m) Rb[m] = 0.5f * (FS[m] - RFtR[m] - RRtF[m]);
}

// Adjoint of w = log_so3(Q) (the literal formula, differentiated by dual
// numbers one entry of Q at a time): Q_bar from w_bar.
__device__ __forceinline__ void rev_log_adjoint(const float Q[9], const float wb[3], float Qb[9]) {
#pragma unroll
  for (int m = 0; m < 9; ++m) {
    Dual<float> Qd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Qd[k] = Dual<float>(Q[k], k == m ? 1.f : 0.f);
    Dual<float> w[3];
    log_so3(Qd, w);
    Qb[m] = wb[0] * w[0].d + wb[1] * w[1].d + wb[2] * w[2].d;
  }
}

__device__ __forceinline__ void rev_items_at(const int64_t *__restrict__ off, int n, int64_t it, int &j, int &a) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= it)
      lo = mid;
    else
      hi = mid - 1;
  }
  j = lo;
  a = (int)(it - off[j]);
}

// Work items of the reverse kernels: one per active sample of every instance
// of the kind that the backward differentiates (prefix sums, n + 1 entries).
__global__ void __launch_bounds__(1024) k_bwd_items_rev(DevBatch b, const InstRec *__restrict__ inst,
                                                        const BwdRec *recs, int kind,
                                                        int64_t *__restrict__ item_off) {
  __shared__ int64_t part[1024];
  const int n = b.n_inst, tid = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int j0 = tid * per, j1 = min(n, j0 + per);
  auto items_of = [&](int j) -> int64_t {
    const BwdRec &r = recs[j];
    const InstRec I = inst[j];
    if (r.status != kBwdOk || I.kind != kind || (I.status & 0xFF) != PURSE_INST_OK ||
        !inst_record_ok(I, inst_view(b, j)))
      return 0;
    return (int64_t)min(max(r.n_act, 0), kMaxActive);
  };
  int64_t acc = 0;
  for (int j = j0; j < j1; ++j) acc += items_of(j);
  part[tid] = acc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int64_t run = tid ? part[tid - 1] : 0;
  for (int j = j0; j < j1; ++j) {
    item_off[j] = run;
    run += items_of(j);
  }
  if (tid == 1023) item_off[n] = part[1023];
}

// The sampler's feasibility test (group-combined).
template <typename T>
__device__ __forceinline__ bool rev_feasible(const KpRec *__restrict__ kp, int n, int q, const float K[4],
                                             const RevPoseT<T> &x, float z_min) {
  bool ok = true;
  for (int i = q; i < n; i += kRevGroup) {
    const KpRec k = kp[i];
    T P[3], iz, u, v;
    project2d(x.R, x.t, k, K, P, iz, u, v);
    const T e0 = u - T(k.c[0]), e1 = v - T(k.c[1]);
    const T et0 = T(k.w[0]) * e0 + T(k.w[1]) * e1, et1 = T(k.w[2]) * e1;
    const T rr = dsqrt(et0 * et0 + et1 * et1);
    ok = ok && (P[2] > T(z_min)) && (rr <= T(k.bt));
  }
  return group_and<kRevGroup>(ok);
}

// One wavefront per kRevSamples active samples; dynamic LDS: the tape,
// kRevSamples x n_iters x n_gn poses of 12 floats.
__global__ void __launch_bounds__(64) k_bwd_rev2d(DevBatch b, DevParams p, const InstRec *__restrict__ inst,
                                                  const KpRec *__restrict__ kprec, const BwdRec *recs,
                                                  const int64_t *__restrict__ item_off,
                                                  const float *__restrict__ tan_all, float *contrib, int max_dirs) {
  extern __shared__ float tape_all[];
  const int64_t total = item_off[b.n_inst];
  const int lane = threadIdx.x, grp = lane / kRevGroup, q = lane % kRevGroup;
  const int passes = p.n_iters * p.n_gn;
  float *tape = tape_all + (int64_t)grp * passes * 12;
  uint8_t *clb = reinterpret_cast<uint8_t *>(tape_all + (int64_t)kRevSamples * (passes > 0 ? passes : 1) * 12) +
                 (int64_t)grp * (p.n_iters > 0 ? p.n_iters : 1) * kRevGroup;
  const float band = ClampBand<Dual<float>>::v;
  for (int64_t wv = blockIdx.x; wv * kRevSamples < total; wv += gridDim.x) {
    const int64_t it = wv * kRevSamples + grp;
    const bool live = it < total;
    int j = 0, a = 0;
    if (live) rev_items_at(item_off, b.n_inst, it, j, a);
    const InstRec I = inst[j];
    const BwdRec *rec = recs + j;
    const KpRec *kp = kprec + I.kp_off;
    const int n = live ? I.n_kp : 0;
    const float oc[3] = {I.oc[0], I.oc[1], I.oc[2]};
    const int s = live ? rec->active[a] : 0;
    // ---------------------------------------------------------- forward
    // The trajectory is recomputed in float64: its decisions (projection
    // clamps, depth, feasibility, bisection) are those of the exact
    // computation, which a float32 recomputation (rounding of a few 1e-6 in
    // r) can take either way for a keypoint converged onto its kink.  The
    // tape keeps the float32 rounding of each pass's input, the clamp bits
    // each iteration's decisions; the sweep below is float32.
    RevPoseT<double> x;
    {
      const PoseT<double> x0 = initial_pose<double>(frame_ref(I), I.seed, (uint64_t)s, p);
#pragma unroll
      for (int m = 0; m < 9; ++m) x.R[m] = x0.R[m];
#pragma unroll
      for (int m = 0; m < 3; ++m) x.t[m] = x0.t[m];
    }
    const double ocd[3] = {I.oc[0], I.oc[1], I.oc[2]};
    bool ok = live;
    for (int itr = 0; itr < p.n_iters && ok; ++itr) {
      const RevPoseT<double> xk = x;
      uint32_t cl = 0u;
      for (int gs = 0; gs < p.n_gn && ok; ++gs) {
        const int ps = itr * p.n_gn + gs;
        if (q < 12) tape[12 * ps + q] = (float)(q < 9 ? x.R[q] : x.t[q - 9]);
        double A[21], g[6], L[21], dinv[6], d[6];
        ok = gs == 0 ? rev_normal_eqs<true, double>(kp, n, q, I.K, ocd, p.z_min, band, xk, x, A, g, cl, false)
                     : rev_normal_eqs<false, double>(kp, n, q, I.K, ocd, p.z_min, band, xk, x, A, g, cl, true);
        ok = ok && chol6_factor<double>(A, L, dinv);
        if (ok) {
          chol6_subst<double>(L, dinv, g, d);
          apply_update<double>(d, ocd, x.R, x.t);
        }
      }
      clb[itr * kRevGroup + q] = (uint8_t)cl;
    }
    const RevPoseT<double> xed = x;  // before the final reorthonormalisation
    reorthonormalise(x.R);
    uint8_t mask = 0;
    float lo = 1.f;
    double wd[3] = {0.0, 0.0, 0.0};
    if (ok) {
      if (rev_feasible<double>(kp, n, q, I.K, x, p.z_min)) {
        mask = PURSE_MASK_FEASIBLE;
      } else if (I.has_anchor) {
        double Rad[9], RaT[9], Q[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Rad[3 * r + c] = I.Ra[3 * r + c];
            RaT[3 * r + c] = I.Ra[3 * c + r];
          }
        matmul3(RaT, x.R, Q);
        log_so3(Q, wd);
        lo = 0.f;
        float hi = 1.f;
        for (int bb = 0; bb < p.n_bis; ++bb) {
          const float mid = 0.5f * (lo + hi);
          const double wm[3] = {mid * wd[0], mid * wd[1], mid * wd[2]};
          double E[9];
          RevPoseT<double> mp;
          exp_so3(wm, E);
          matmul3(Rad, E, mp.R);
#pragma unroll
          for (int r = 0; r < 3; ++r) mp.t[r] = (double)I.ta[r] + mid * (x.t[r] - (double)I.ta[r]);
          if (rev_feasible<double>(kp, n, q, I.K, mp, p.z_min))
            lo = mid;
          else
            hi = mid;
        }
        mask = PURSE_MASK_FEASIBLE | PURSE_MASK_PULLED_IN;
      }
    }
    RevPose xf, xe;
    rev_round(x, xf);
    rev_round(xed, xe);
    const float w[3] = {(float)wd[0], (float)wd[1], (float)wd[2]};
    __syncthreads();  // the tape is complete
    // ---------------------------------------------------------- reverse
    float Rcb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, tcb[3] = {0.f, 0.f, 0.f};
    float Rab[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, tab[3] = {0.f, 0.f, 0.f};
    float ob_u[3] = {0.f, 0.f, 0.f};
    float kb[kRevPerLane][6];
#pragma unroll
    for (int rr = 0; rr < kRevPerLane; ++rr)
#pragma unroll
      for (int m = 0; m < 6; ++m) kb[rr][m] = 0.f;
    if (mask & PURSE_MASK_FEASIBLE) {
      float cR[9], ct[3];
#pragma unroll
      for (int m = 0; m < 9; ++m) cR[m] = (float)rec->cot[a][m];
#pragma unroll
      for (int m = 0; m < 3; ++m) ct[m] = (float)rec->cot[a][9 + m];
      RevPose xb;
      if (!(mask & PURSE_MASK_PULLED_IN)) {
#pragma unroll
        for (int m = 0; m < 9; ++m) xb.R[m] = cR[m];
#pragma unroll
        for (int m = 0; m < 3; ++m) xb.t[m] = ct[m];
      } else if (lo == 0.f) {
        // the anchor itself
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          Rab[m] += cR[m];
          xb.R[m] = 0.f;
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          tab[m] += ct[m];
          xb.t[m] = 0.f;
        }
      } else {
        // out = (Ra Exp(lo w), ta + lo (t - ta)), w = Log(Ra^T R)
        const float phi[3] = {lo * w[0], lo * w[1], lo * w[2]};
        float E[9], Eb[9], phib[3], Qb[9], RaT[9], Q[9];
        exp_so3(phi, E);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Rab[3 * r + c] += cR[3 * r] * E[3 * c] + cR[3 * r + 1] * E[3 * c + 1] + cR[3 * r + 2] * E[3 * c + 2];
            Eb[3 * r + c] = I.Ra[r] * cR[c] + I.Ra[3 + r] * cR[3 + c] + I.Ra[6 + r] * cR[6 + c];
            RaT[3 * r + c] = I.Ra[3 * c + r];
          }
        rev_exp_adjoint(phi, Eb, phib);
        const float wb[3] = {lo * phib[0], lo * phib[1], lo * phib[2]};
        matmul3(RaT, xf.R, Q);
        rev_log_adjoint(Q, wb, Qb);
        // Q = Ra^T R: R_bar = Ra Q_bar, Ra_bar += R Q_bar^T
        matmul3(I.Ra, Qb, xb.R);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            Rab[3 * r + c] += xf.R[3 * r] * Qb[3 * c] + xf.R[3 * r + 1] * Qb[3 * c + 1] + xf.R[3 * r + 2] * Qb[3 * c + 2];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          xb.t[m] = lo * ct[m];
          tab[m] += (1.f - lo) * ct[m];
        }
      }
      rev_reorthonormalise(xe.R, xb.R);
      for (int itr = p.n_iters - 1; itr >= 0; --itr) {
        RevPose xk, xkb;
        const float *tk = tape + 12 * (itr * p.n_gn);
        const uint32_t clbi = clb[itr * kRevGroup + q];
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          xk.R[m] = tk[m];
          xkb.R[m] = 0.f;
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          xk.t[m] = tk[9 + m];
          xkb.t[m] = 0.f;
        }
        for (int gs = p.n_gn - 1; gs >= 1; --gs) {
          const float *tx = tape + 12 * (itr * p.n_gn + gs);
          RevPose xin;
#pragma unroll
          for (int m = 0; m < 9; ++m) xin.R[m] = tx[m];
#pragma unroll
          for (int m = 0; m < 3; ++m) xin.t[m] = tx[9 + m];
          rev_pass<false>(kp, n, q, I.K, oc, p.z_min, clbi, xk, xin, xb, xkb, ob_u, kb);
        }
        rev_pass<true>(kp, n, q, I.K, oc, p.z_min, clbi, xk, xk, xb, xkb, ob_u, kb);
      }
      // the start: even s rotate the centre by E about the pivot, odd s shift it
      if ((s & 1) == 0) {
        float dd[3];
        trajectory_direction(I.seed, (uint64_t)s, dd);
        const float w0[3] = {p.omega0 * dd[0], p.omega0 * dd[1], p.omega0 * dd[2]};
        float E[9];
        exp_so3(w0, E);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            Rcb[3 * r + c] += E[r] * xb.R[c] + E[3 + r] * xb.R[3 + c] + E[6 + r] * xb.R[6 + c];
          const float et = E[r] * xb.t[0] + E[3 + r] * xb.t[1] + E[6 + r] * xb.t[2];
          tcb[r] += et;
          ob_u[r] += xb.t[r] - et;
        }
      } else {
#pragma unroll
        for (int m = 0; m < 9; ++m) Rcb[m] += xb.R[m];
#pragma unroll
        for (int m = 0; m < 3; ++m) tcb[m] += xb.t[m];
      }
    }
    float fb[27];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      fb[m] = Rcb[m];
      fb[15 + m] = Rab[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      fb[9 + m] = tcb[m];
      fb[12 + m] = ob_u[m];
      fb[24 + m] = tab[m];
    }
    // ---------------------------------------------------- contributions
    if (live) {
      const bool feas = (mask & PURSE_MASK_FEASIBLE) != 0;
#pragma unroll
      for (int rr = 0; rr < kRevPerLane; ++rr) {
        const int i = q + kRevGroup * rr;
        if (i >= n) break;
        for (int c = 0; c < 6; ++c) {
          const int d = 6 * i + c;
          float acc = 0.f;
          if (feas) {
            KpT<Dual<float>> tk;
            kp_tangent(I, kp[i], b.shapes + 4 * (I.kp_off + i), b.bounds[I.kp_off + i], p.kappa, c, tk);
            acc = kb[rr][0] * tk.c[0].d + kb[rr][1] * tk.c[1].d + kb[rr][2] * tk.w[0].d + kb[rr][3] * tk.w[1].d +
                  kb[rr][4] * tk.w[2].d + kb[rr][5] * tk.kb.d;
            const float *tn = tan_all + ((int64_t)j * max_dirs + d) * 27;
#pragma unroll
            for (int m = 0; m < 27; ++m) acc += fb[m] * tn[m];
          }
          contrib[((int64_t)j * kMaxActive + a) * max_dirs + d] = acc;
        }
      }
    }
    __syncthreads();  // (the next samples' forward rewrites the tape)
  }
}

// ---------------------------------------------------------------------------
// 3D-3D reverse sweep.  One iteration of the refit from x = (R, t):
//   tt = t + R abar; per keypoint d = tt - c, e = R m + d, s = kappa beta / |e|
//   when clamped (else 1), q = s e - d; M = sum q m^T, qs = sum q;
//   R' = proj_SO3(M), t' = tt + qs / N - R' abar.
// Its adjoint, from (R'_bar, t'_bar): tt_bar = t'_bar, qs_bar = t'_bar / N and
// R'_bar - t'_bar abar^T into the polar factor, whose adjoint is
// M_bar = R' [y]x with (tr(S) I - S) y = vee(R'^T R'_bar - R'_bar^T R'),
// S = R'^T M (differentiating M = R' S with S symmetric and R'^T dR' skew,
// then moving the symmetric operator Omega -> Omega S + S Omega across the
// inner product); per keypoint q_bar = M_bar m + qs_bar, e_bar = s q_bar
// (plus 2 r2_bar e and kappa_beta_bar += s_bar / |e| when clamped, with
// s_bar = q_bar . e and r2_bar = -s_bar s / (2 |e|^2)), d_bar = e_bar - q_bar,
// R_bar += e_bar m^T, tt_bar += d_bar, c_bar -= d_bar; finally t_bar = tt_bar
// and R_bar += tt_bar abar^T.  Same lane groups and tape as the 2D-3D sweep
// (one pose per iteration), the same frozen decisions.

// Group-summed M and qs of one iteration at x, and tt; projection decisions
// in cl as in rev_normal_eqs (taken from cl when use_cl, else recorded).
template <typename T>
__device__ __forceinline__ void rev3d_sums(const KpRec *__restrict__ kp, int n, int q, const float abar[3],
                                           float band, const RevPoseT<T> &x, T tt[3], T M[9], T qs[3],
                                           uint32_t &cl, bool use_cl) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    tt[r] = x.t[r] + x.R[3 * r] * T(abar[0]) + x.R[3 * r + 1] * T(abar[1]) + x.R[3 * r + 2] * T(abar[2]);
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) qs[k] = T(0);
  if (!use_cl) cl = 0u;
  for (int i = q, rr = 0; i < n; i += kRevGroup, ++rr) {
    const KpRec k = kp[i];
    T d[3], e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      d[r] = tt[r] - T(k.c[r]);
      e[r] = x.R[3 * r] * T(k.m[0]) + x.R[3 * r + 1] * T(k.m[1]) + x.R[3 * r + 2] * T(k.m[2]) + d[r];
    }
    const T r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    if (!use_cl && !(r2 <= T(k.kb2) * T(band))) cl |= 1u << rr;
    const T sc = ((cl >> rr) & 1u) ? T(k.kb) * drsqrt(r2) : T(1);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const T qq = sc * e[r] - d[r];
      M[3 * r] += qq * T(k.m[0]);
      M[3 * r + 1] += qq * T(k.m[1]);
      M[3 * r + 2] += qq * T(k.m[2]);
      qs[r] += qq;
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = group_sum<kRevGroup>(M[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) qs[k] = group_sum<kRevGroup>(qs[k]);
}

// M_bar of R = proj_SO3(M) from R_bar (R the computed factor).
__device__ __forceinline__ void rev_polar_adjoint(const float M[9], const float R[9], const float Rb[9],
                                                  float Mb[9]) {
  float S[9], X[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      S[3 * r + c] = R[r] * M[c] + R[3 + r] * M[3 + c] + R[6 + r] * M[6 + c];
      X[3 * r + c] = R[r] * Rb[c] + R[3 + r] * Rb[3 + c] + R[6 + r] * Rb[6 + c];
    }
  const float a[3] = {X[7] - X[5], X[2] - X[6], X[3] - X[1]};
  // B = tr(S) I - sym(S), solved by its adjugate
  const float tr = S[0] + S[4] + S[8];
  const float b00 = tr - S[0], b11 = tr - S[4], b22 = tr - S[8];
  const float b01 = -0.5f * (S[1] + S[3]), b02 = -0.5f * (S[2] + S[6]), b12 = -0.5f * (S[5] + S[7]);
  const float c00 = b11 * b22 - b12 * b12, c01 = b02 * b12 - b01 * b22, c02 = b01 * b12 - b02 * b11;
  const float c11 = b00 * b22 - b02 * b02, c12 = b01 * b02 - b00 * b12, c22 = b00 * b11 - b01 * b01;
  const float idet = 1.f / (b00 * c00 + b01 * c01 + b02 * c02);
  const float y[3] = {(c00 * a[0] + c01 * a[1] + c02 * a[2]) * idet, (c01 * a[0] + c11 * a[1] + c12 * a[2]) * idet,
                      (c02 * a[0] + c12 * a[1] + c22 * a[2]) * idet};
  // M_bar = R [y]x
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Mb[3 * r] = R[3 * r + 1] * y[2] - R[3 * r + 2] * y[1];
    Mb[3 * r + 1] = R[3 * r + 2] * y[0] - R[3 * r] * y[2];
    Mb[3 * r + 2] = R[3 * r] * y[1] - R[3 * r + 1] * y[0];
  }
}

// One iteration of the reverse sweep: xb holds the cotangent of the
// iteration's output (whose rotation is Rn) on entry and of its input x on
// return; the keypoints' cotangents (c_bar in kb[.][0..2], kappa beta in
// kb[.][3]) accumulate per lane.
__device__ __forceinline__ void rev3d_iter(const KpRec *__restrict__ kp, int n, int q, const float abar[3],
                                           uint32_t clbits, const RevPose &x, const float Rn[9], RevPose &xb,
                                           float kb[kRevPerLane][6]) {
  float tt[3], M[9], qs[3];
  rev3d_sums<float>(kp, n, q, abar, 1.f, x, tt, M, qs, clbits, true);
  const float inv_n = 1.f / (float)n;
  float qsb[3], Rpb[9], Mb[9];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    qsb[r] = xb.t[r] * inv_n;
#pragma unroll
    for (int c = 0; c < 3; ++c) Rpb[3 * r + c] = xb.R[3 * r + c] - xb.t[r] * abar[c];
  }
  rev_polar_adjoint(M, Rn, Rpb, Mb);
  float Rbp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, ttbp[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int rr = 0; rr < kRevPerLane; ++rr) {
    const int i = q + kRevGroup * rr;
    if (i >= n) break;
    const KpRec k = kp[i];
    float d[3], e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      d[r] = tt[r] - k.c[r];
      e[r] = x.R[3 * r] * k.m[0] + x.R[3 * r + 1] * k.m[1] + x.R[3 * r + 2] * k.m[2] + d[r];
    }
    const float r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    const bool cl = (clbits >> rr) & 1u;
    const float sc = cl ? k.kb * drsqrt(r2) : 1.f;
    float qb[3], eb[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      qb[r] = Mb[3 * r] * k.m[0] + Mb[3 * r + 1] * k.m[1] + Mb[3 * r + 2] * k.m[2] + qsb[r];
      eb[r] = sc * qb[r];
    }
    if (cl) {
      const float sb = qb[0] * e[0] + qb[1] * e[1] + qb[2] * e[2];
      kb[rr][3] += sb * drsqrt(r2);
      const float r2b = -0.5f * sb * sc / r2;
#pragma unroll
      for (int r = 0; r < 3; ++r) eb[r] += 2.f * r2b * e[r];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float db = eb[r] - qb[r];
      Rbp[3 * r] += eb[r] * k.m[0];
      Rbp[3 * r + 1] += eb[r] * k.m[1];
      Rbp[3 * r + 2] += eb[r] * k.m[2];
      ttbp[r] += db;
      kb[rr][r] -= db;
    }
  }
  float ttb[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) ttb[r] = xb.t[r] + group_sum<kRevGroup>(ttbp[r]);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    xb.t[r] = ttb[r];
#pragma unroll
    for (int c = 0; c < 3; ++c) xb.R[3 * r + c] = group_sum<kRevGroup>(Rbp[3 * r + c]) + ttb[r] * abar[c];
  }
}

// The sampler's 3D-3D feasibility test (group-combined).
template <typename T>
__device__ __forceinline__ bool rev3d_feasible(const KpRec *__restrict__ kp, int n, int q, const float abar[3],
                                               const RevPoseT<T> &x) {
  T tt[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    tt[r] = x.t[r] + x.R[3 * r] * T(abar[0]) + x.R[3 * r + 1] * T(abar[1]) + x.R[3 * r + 2] * T(abar[2]);
  bool ok = true;
  for (int i = q; i < n; i += kRevGroup) {
    const KpRec k = kp[i];
    T e[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      e[r] = x.R[3 * r] * T(k.m[0]) + x.R[3 * r + 1] * T(k.m[1]) + x.R[3 * r + 2] * T(k.m[2]) + tt[r] - T(k.c[r]);
    ok = ok && (dsqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]) <= T(k.bt));
  }
  return group_and<kRevGroup>(ok);
}

// One wavefront per kRevSamples active samples of 3D-3D instances; dynamic
// LDS: the tape, kRevSamples x n_iters poses of 12 floats.
__global__ void __launch_bounds__(64) k_bwd_rev3d(DevBatch b, DevParams p, const InstRec *__restrict__ inst,
                                                  const KpRec *__restrict__ kprec, const BwdRec *recs,
                                                  const int64_t *__restrict__ item_off,
                                                  const float *__restrict__ tan_all, float *contrib, int max_dirs) {
  extern __shared__ float tape_all[];
  const int64_t total = item_off[b.n_inst];
  const int lane = threadIdx.x, grp = lane / kRevGroup, q = lane % kRevGroup;
  const int iters = p.n_iters;
  const int it_alloc = iters > 0 ? iters : 1;
  float *tape = tape_all + (int64_t)grp * it_alloc * 12;
  uint8_t *clb = reinterpret_cast<uint8_t *>(tape_all + (int64_t)kRevSamples * it_alloc * 12) +
                 (int64_t)grp * it_alloc * kRevGroup;
  const float band = ClampBand<Dual<float>>::v;
  for (int64_t wv = blockIdx.x; wv * kRevSamples < total; wv += gridDim.x) {
    const int64_t it = wv * kRevSamples + grp;
    const bool live = it < total;
    int j = 0, a = 0;
    if (live) rev_items_at(item_off, b.n_inst, it, j, a);
    const InstRec I = inst[j];
    const BwdRec *rec = recs + j;
    const KpRec *kp = kprec + I.kp_off;
    const int n = live ? I.n_kp : 0;
    const int s = live ? rec->active[a] : 0;
    // ---------------------------------------------------------- forward
    // In float64, as in the 2D-3D sweep (the polar factor by the float64
    // Jacobi iteration); float32 tape and clamp bits for the sweep.
    RevPoseT<double> x;
    {
      const PoseT<double> x0 = initial_pose<double>(frame_ref(I), I.seed, (uint64_t)s, p);
#pragma unroll
      for (int m = 0; m < 9; ++m) x.R[m] = x0.R[m];
#pragma unroll
      for (int m = 0; m < 3; ++m) x.t[m] = x0.t[m];
    }
    if (live) {
      const double inv_n = 1.0 / (double)n;
      for (int itr = 0; itr < iters; ++itr) {
        if (q < 12) tape[12 * itr + q] = (float)(q < 9 ? x.R[q] : x.t[q - 9]);
        double tt[3], M[9], qs[3];
        uint32_t cl = 0u;
        rev3d_sums<double>(kp, n, q, I.abar, band, x, tt, M, qs, cl, false);
        clb[itr * kRevGroup + q] = (uint8_t)cl;
        polar_so3<double>(M, x.R, 10);
#pragma unroll
        for (int r = 0; r < 3; ++r)
          x.t[r] = tt[r] + qs[r] * inv_n -
                   (x.R[3 * r] * (double)I.abar[0] + x.R[3 * r + 1] * (double)I.abar[1] +
                    x.R[3 * r + 2] * (double)I.abar[2]);
      }
    }
    uint8_t mask = 0;
    float lo = 1.f;
    double wd[3] = {0.0, 0.0, 0.0};
    if (live) {
      if (rev3d_feasible<double>(kp, n, q, I.abar, x)) {
        mask = PURSE_MASK_FEASIBLE;
      } else if (I.has_anchor) {
        double Rad[9], RaT[9], Q[9];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Rad[3 * r + c] = I.Ra[3 * r + c];
            RaT[3 * r + c] = I.Ra[3 * c + r];
          }
        matmul3(RaT, x.R, Q);
        log_so3(Q, wd);
        lo = 0.f;
        float hi = 1.f;
        for (int bb = 0; bb < p.n_bis; ++bb) {
          const float mid = 0.5f * (lo + hi);
          const double wm[3] = {mid * wd[0], mid * wd[1], mid * wd[2]};
          double E[9];
          RevPoseT<double> mp;
          exp_so3(wm, E);
          matmul3(Rad, E, mp.R);
#pragma unroll
          for (int r = 0; r < 3; ++r) mp.t[r] = (double)I.ta[r] + mid * (x.t[r] - (double)I.ta[r]);
          if (rev3d_feasible<double>(kp, n, q, I.abar, mp))
            lo = mid;
          else
            hi = mid;
        }
        mask = PURSE_MASK_FEASIBLE | PURSE_MASK_PULLED_IN;
      }
    }
    RevPose xf;
    rev_round(x, xf);
    const float w[3] = {(float)wd[0], (float)wd[1], (float)wd[2]};
    __syncthreads();  // the tape is complete
    // ---------------------------------------------------------- reverse
    float Rcb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, tcb[3] = {0.f, 0.f, 0.f};
    float Rab[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, tab[3] = {0.f, 0.f, 0.f};
    float ob_u[3] = {0.f, 0.f, 0.f};
    float kb[kRevPerLane][6];
#pragma unroll
    for (int rr = 0; rr < kRevPerLane; ++rr)
#pragma unroll
      for (int m = 0; m < 6; ++m) kb[rr][m] = 0.f;
    if (mask & PURSE_MASK_FEASIBLE) {
      float cR[9], ct[3];
#pragma unroll
      for (int m = 0; m < 9; ++m) cR[m] = (float)rec->cot[a][m];
#pragma unroll
      for (int m = 0; m < 3; ++m) ct[m] = (float)rec->cot[a][9 + m];
      RevPose xb;
      if (!(mask & PURSE_MASK_PULLED_IN)) {
#pragma unroll
        for (int m = 0; m < 9; ++m) xb.R[m] = cR[m];
#pragma unroll
        for (int m = 0; m < 3; ++m) xb.t[m] = ct[m];
      } else if (lo == 0.f) {
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          Rab[m] += cR[m];
          xb.R[m] = 0.f;
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          tab[m] += ct[m];
          xb.t[m] = 0.f;
        }
      } else {
        // out = (Ra Exp(lo w), ta + lo (t - ta)), w = Log(Ra^T R)
        const float phi[3] = {lo * w[0], lo * w[1], lo * w[2]};
        float E[9], Eb[9], phib[3], Qb[9], RaT[9], Q[9];
        exp_so3(phi, E);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Rab[3 * r + c] += cR[3 * r] * E[3 * c] + cR[3 * r + 1] * E[3 * c + 1] + cR[3 * r + 2] * E[3 * c + 2];
            Eb[3 * r + c] = I.Ra[r] * cR[c] + I.Ra[3 + r] * cR[3 + c] + I.Ra[6 + r] * cR[6 + c];
            RaT[3 * r + c] = I.Ra[3 * c + r];
          }
        rev_exp_adjoint(phi, Eb, phib);
        const float wb[3] = {lo * phib[0], lo * phib[1], lo * phib[2]};
        matmul3(RaT, xf.R, Q);
        rev_log_adjoint(Q, wb, Qb);
        matmul3(I.Ra, Qb, xb.R);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c)
            Rab[3 * r + c] += xf.R[3 * r] * Qb[3 * c] + xf.R[3 * r + 1] * Qb[3 * c + 1] + xf.R[3 * r + 2] * Qb[3 * c + 2];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          xb.t[m] = lo * ct[m];
          tab[m] += (1.f - lo) * ct[m];
        }
      }
      for (int itr = iters - 1; itr >= 0; --itr) {
        RevPose xin;
        float Rn[9];
        const float *tx = tape + 12 * itr;
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          xin.R[m] = tx[m];
          Rn[m] = itr + 1 < iters ? tx[12 + m] : xf.R[m];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) xin.t[m] = tx[9 + m];
        rev3d_iter(kp, n, q, I.abar, clb[itr * kRevGroup + q], xin, Rn, xb, kb);
      }
      // the start: even s rotate the centre by E about the pivot, odd s shift it
      if ((s & 1) == 0) {
        float dd[3];
        trajectory_direction(I.seed, (uint64_t)s, dd);
        const float w0[3] = {p.omega0 * dd[0], p.omega0 * dd[1], p.omega0 * dd[2]};
        float E[9];
        exp_so3(w0, E);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            Rcb[3 * r + c] += E[r] * xb.R[c] + E[3 + r] * xb.R[3 + c] + E[6 + r] * xb.R[6 + c];
          const float et = E[r] * xb.t[0] + E[3 + r] * xb.t[1] + E[6 + r] * xb.t[2];
          tcb[r] += et;
          ob_u[r] += xb.t[r] - et;
        }
      } else {
#pragma unroll
        for (int m = 0; m < 9; ++m) Rcb[m] += xb.R[m];
#pragma unroll
        for (int m = 0; m < 3; ++m) tcb[m] += xb.t[m];
      }
    }
    float fb[27];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      fb[m] = Rcb[m];
      fb[15 + m] = Rab[m];
    }
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      fb[9 + m] = tcb[m];
      fb[12 + m] = ob_u[m];
      fb[24 + m] = tab[m];
    }
    // ---------------------------------------------------- contributions
    if (live) {
      const bool feas = (mask & PURSE_MASK_FEASIBLE) != 0;
      const int dpk = dirs_per_kp(PURSE_KIND_3D3D);
#pragma unroll
      for (int rr = 0; rr < kRevPerLane; ++rr) {
        const int i = q + kRevGroup * rr;
        if (i >= n) break;
        for (int c = 0; c < dpk; ++c) {
          const int d = dpk * i + c;
          float acc = 0.f;
          if (feas) {
            KpT<Dual<float>> tk;
            kp_tangent(I, kp[i], b.shapes + 4 * (I.kp_off + i), b.bounds[I.kp_off + i], p.kappa, c, tk);
            acc = kb[rr][0] * tk.c[0].d + kb[rr][1] * tk.c[1].d + kb[rr][2] * tk.c[2].d + kb[rr][3] * tk.kb.d;
            const float *tn = tan_all + ((int64_t)j * max_dirs + d) * 27;
#pragma unroll
            for (int m = 0; m < 27; ++m) acc += fb[m] * tn[m];
          }
          contrib[((int64_t)j * kMaxActive + a) * max_dirs + d] = acc;
        }
      }
    }
    __syncthreads();  // (the next samples' forward rewrites the tape)
  }
}

// Sum over active samples (fixed order) and scatter into the gradients.
__global__ void __launch_bounds__(kMaxDirs) k_bwd_reduce(DevBatch b, const InstRec *__restrict__ inst,
                                                        const BwdRec *recs, const float *__restrict__ contrib,
                                                        int max_dirs, float *g_centres, float *g_shapes,
                                                        float *g_bounds, int32_t *bwd_status) {
  const int j = blockIdx.x;
  const int d = threadIdx.x;
  if (d == 0 && bwd_status) bwd_status[j] = recs[j].status | (min(recs[j].n_distinct, 0xFFFFFF) << 8);
  const InstView v = inst_view(b, j);
  if (!inst_view_ok(v)) return;  // (the batch's own ranges: nothing can be addressed)
  const int64_t ko = v.kp_off;
  const int n = v.n_kp;
  const bool is2d = v.kind == PURSE_KIND_2D3D;
  const int dpk = dirs_per_kp(v.kind);
  if (d >= n * dpk) return;
  const int i = d / dpk, c = d % dpk;
  const InstRec I = inst[j];
  const BwdRec *rec = recs + j;
  float g = 0.f;
  if (bwd_status_is_error(rec->status) || !inst_record_ok(I, v)) {
    // a stale workspace, an active set beyond capacity, a trace that does not
    // fit the mask, or a non-finite centre: no gradient
    g = __int_as_float(0x7fc00000);
  } else if ((I.status & 0xFF) == PURSE_INST_OK && rec->status == kBwdOk) {
    double acc = 0.0;
    const int n_act = min(max(rec->n_act, 0), kMaxActive);  // (the record's capacity)
    for (int a = 0; a < n_act; ++a) acc += (double)contrib[((int64_t)j * kMaxActive + a) * max_dirs + d];
    g = (float)acc;
  }
  const int64_t k = ko + i;
  if (c == 0) {
    if (is2d)
      g_centres[3 * k + 2] = 0.f;
    else
      for (int q = 0; q < 4; ++q) g_shapes[4 * k + q] = 0.f;
  }
  if (is2d) {
    if (c < 2)
      g_centres[3 * k + c] = g;
    else if (c == 2)
      g_shapes[4 * k] = g;
    else if (c == 3) {
      g_shapes[4 * k + 1] = 0.5f * g;
      g_shapes[4 * k + 2] = 0.5f * g;
    } else if (c == 4)
      g_shapes[4 * k + 3] = g;
    else
      g_bounds[k] = g;
  } else {
    if (c < 3)
      g_centres[3 * k + c] = g;
    else
      g_bounds[k] = g;
  }
}

namespace {

// One auxiliary stream (default priority) and two events per device, created
// on first use and kept until the process ends.
struct Aux {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_aux_mu;
Aux g_aux[64];

Aux *aux_stream() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  Aux &a = g_aux[dev];
  if (!a.s) {
    hipStream_t s = nullptr;
    hipEvent_t f = nullptr, jn = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (hipEventCreateWithFlags(&f, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&jn, hipEventDisableTiming) != hipSuccess) {
      if (f) (void)hipEventDestroy(f);
      (void)hipStreamDestroy(s);
      return nullptr;
    }
    a.s = s;
    a.fork = f;
    a.join = jn;
  }
  return &a;
}

}  // namespace

hipError_t launch_backward(const DevBatch &b, const DevParams &p, const float *poses, const uint8_t *mask,
                           const int32_t *trace, const double *g_radii, const float *g_centre, const InstRec *inst,
                           const KpRec *kp, MegbRec *megb, BwdRec *recs, float4 *ckpt, float *tan, float *contrib,
                           int64_t *items, float *g_centres, float *g_shapes, float *g_bounds, int32_t *bwd_status,
                           hipStream_t stream) {
  const int n = b.n_inst;
  const int ck = ckpt_spacing(p.ckpt_every);
  const int max_dirs = 6 * b.max_kp;
  // k_bwd_frame on the device's auxiliary stream, concurrently with
  // k_bwd_megb (a fork and a join by events, which graph capture records as
  // edges); on the caller's stream when there is none
  {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    Aux *a = aux_stream();
    if (a && hipEventRecord(a->fork, stream) == hipSuccess && hipStreamWaitEvent(a->s, a->fork, 0) == hipSuccess) {
      hipLaunchKernelGGL(k_bwd_frame, dim3(n), dim3(kMaxDirs), 0, a->s, b, p, inst, kp, tan, max_dirs);
      hipError_t e = hipEventRecord(a->join, a->s);
      hipLaunchKernelGGL(k_bwd_megb, dim3(n), dim3(kBwdBlock), 0, stream, b, p, poses, mask, trace, g_radii,
                         g_centre, inst, megb, recs, ckpt, ck);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, a->join, 0);
      if (e != hipSuccess) return e;  // no join: nothing that reads the frame tangents is launched
    } else {
      hipLaunchKernelGGL(k_bwd_megb, dim3(n), dim3(kBwdBlock), 0, stream, b, p, poses, mask, trace, g_radii,
                         g_centre, inst, megb, recs, ckpt, ck);
      hipLaunchKernelGGL(k_bwd_frame, dim3(n), dim3(kMaxDirs), 0, stream, b, p, inst, kp, tan, max_dirs);
    }
  }
  // the tangent kernels walk lists of the (instance, active sample,
  // direction block) items the active sets need: the 2D-3D ones on the
  // caller's stream and the 3D-3D ones on the auxiliary stream beside them
  // (they touch disjoint items and contributions), joined before the
  // reduction
  std::unique_lock<std::mutex> lk(g_aux_mu);
  Aux *a = aux_stream();
  const bool fork = a && hipEventRecord(a->fork, stream) == hipSuccess &&
                    hipStreamWaitEvent(a->s, a->fork, 0) == hipSuccess;
  if (!fork) lk.unlock();
  hipStream_t s3 = fork ? a->s : stream;
  // 2D-3D: one reverse sweep per active sample while the tape fits in LDS,
  // else (or when asked) one forward-mode re-run per input direction
  const int passes = p.n_iters * p.n_gn;
  const size_t lds2 = rev_lds(passes, p.n_iters);
  const bool reverse = lds2 <= kRevLds && !(p.flags & PURSE_FLAG_FORWARD_TANGENTS);
  if (reverse) {
    hipLaunchKernelGGL(k_bwd_items_rev, dim3(1), dim3(1024), 0, stream, b, inst, recs, (int)PURSE_KIND_2D3D, items);
    const size_t lds = lds2;
    hipLaunchKernelGGL(k_bwd_rev2d, dim3(kItemGrid), dim3(64), lds, stream, b, p, inst, kp, recs, items, tan,
                       contrib, max_dirs);
  } else {
    hipLaunchKernelGGL(k_bwd_items, dim3(1), dim3(1024), 0, stream, b, inst, recs, (int)PURSE_KIND_2D3D, kTrajGroup,
                       items);
    hipLaunchKernelGGL(k_bwd_traj2d_group<kTrajGroup>, dim3(kItemGrid), dim3(64), 0, stream, b, p, inst, kp, recs,
                       items, tan, contrib, max_dirs);
  }
  // 3D-3D likewise, with one tape pose per iteration
  const size_t lds3 = rev_lds(p.n_iters, p.n_iters);
  const bool reverse3 = lds3 <= kRevLds && !(p.flags & PURSE_FLAG_FORWARD_TANGENTS);
  if (reverse3) {
    hipLaunchKernelGGL(k_bwd_items_rev, dim3(1), dim3(1024), 0, s3, b, inst, recs, (int)PURSE_KIND_3D3D,
                       items + (n + 1));
    const size_t lds = lds3;
    hipLaunchKernelGGL(k_bwd_rev3d, dim3(kItemGrid), dim3(64), lds, s3, b, p, inst, kp, recs, items + (n + 1),
                       tan, contrib, max_dirs);
  } else {
    hipLaunchKernelGGL(k_bwd_items, dim3(1), dim3(1024), 0, s3, b, inst, recs, (int)PURSE_KIND_3D3D, 1,
                       items + (n + 1));
    hipLaunchKernelGGL(k_bwd_traj<PURSE_KIND_3D3D>, dim3(kItemGrid), dim3(64), 0, s3, b, p, inst, kp, recs,
                       items + (n + 1), tan, contrib, max_dirs);
  }
  if (fork) {
    hipError_t e = hipEventRecord(a->join, a->s);
    if (e == hipSuccess) e = hipStreamWaitEvent(stream, a->join, 0);
    if (e != hipSuccess) return e;  // no join: the reduction is not launched
  }
  hipLaunchKernelGGL(k_bwd_reduce, dim3(n), dim3(kMaxDirs), 0, stream, b, inst, recs, contrib, max_dirs, g_centres,
                     g_shapes, g_bounds, bwd_status);
  return hipSuccess;
}

}  // namespace purse
