// Checks the backward applies before any workspace record or data-derived
// value becomes a memory index: the prologue's records must belong to the
// batch given, every sample id must lie in its instance's range, and the
// active-set bookkeeping must stay within its capacity.  Host and device
// share these functions, so the host test that drives them with stale
// records, non-finite centres and out-of-range ids exercises the code the
// kernels run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "purse_layout.hpp"

namespace purse {

// BwdRec.status values
constexpr int32_t kBwdOk = 0;
constexpr int32_t kBwdEmpty = 1;        // no feasible sample: zero gradients
constexpr int32_t kBwdOverflow = 2;     // the descent touched more than kMaxActive samples
constexpr int32_t kBwdBadTrace = 3;     // a trace entry is no feasible sample of the instance
constexpr int32_t kBwdStale = 4;        // the workspace records belong to another batch or data
constexpr int32_t kBwdNonFinite = 5;    // the centre is not finite: no radius sample exists

// True when a BwdRec status means "no gradient" (NaN) rather than zero.
__host__ __device__ inline bool bwd_status_is_error(int32_t s) { return s != kBwdOk && s != kBwdEmpty; }

// Instance j of the batch as the backward sees it (values read from the
// caller's batch arrays).
struct InstView {
  int32_t kind, n_kp;
  int64_t kp_off, kp_end;     // kp_off[j], kp_off[j + 1]
  int64_t s_off, s_end;       // sample_off[j], sample_off[j + 1]
  uint64_t seed;
  int64_t total_kp, total_samples, max_samples;
};

__device__ inline InstView inst_view(const DevBatch &b, int j) {
  InstView v;
  v.kind = b.kind[j];
  v.n_kp = b.n_kp[j];
  v.kp_off = b.kp_off[j];
  v.kp_end = b.kp_off[j + 1];
  v.s_off = b.sample_off[j];
  v.s_end = b.sample_off[j + 1];
  v.seed = b.seed[j];
  v.total_kp = b.total_kp;
  v.total_samples = b.total_samples;
  v.max_samples = b.max_samples;
  return v;
}

// The batch's own description of instance j is self-consistent: its
// keypoint range (at most PURSE_MAX_KP keypoints) and sample range lie inside
// the arrays.  (Whether the instance is valid for the method is the
// prologue's status, not this.)
__host__ __device__ inline bool inst_view_ok(const InstView &v) {
  return v.n_kp >= 0 && v.n_kp <= PURSE_MAX_KP && v.kp_off >= 0 && v.kp_end - v.kp_off == (int64_t)v.n_kp &&
         v.kp_end <= v.total_kp && v.s_off >= 0 && v.s_end >= v.s_off && v.s_end - v.s_off <= v.max_samples &&
         v.s_end <= v.total_samples;
}

// The prologue's record describes instance j of this batch: same kind,
// keypoint range, sample range and Philox key, and a valid batch entry.
// Every backward kernel checks this before it uses a record field as an
// offset.
__host__ __device__ inline bool inst_record_ok(const InstRec &I, const InstView &v) {
  return inst_view_ok(v) && I.kind == v.kind && I.n_kp == v.n_kp && I.kp_off == v.kp_off &&
         I.sample_off == v.s_off && I.n_samples == v.s_end - v.s_off && I.seed == v.seed;
}

// 64-bit mix (splitmix64 finaliser)
__host__ __device__ inline unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Fingerprint term of keypoint i's measurements (centre, shape, bound) and
// model point: summed (wrapping) over the keypoints, so the sum does not
// depend on order.  The prologue stores the sum in the instance record; the
// backward recomputes it from the batch it is given.
__host__ __device__ inline unsigned long long kp_data_term(int i, const uint32_t w[11]) {
  unsigned long long z = mix64(0x5055525345ull + (unsigned long long)(unsigned)i);
  for (int k = 0; k < 11; ++k) z = mix64(z ^ ((unsigned long long)w[k] << (k & 1 ? 32 : 0)));
  return z;
}

__host__ __device__ inline uint32_t fbits(float x) { return __builtin_bit_cast(uint32_t, x); }

// The 11 words of keypoint i that the fingerprint covers: model point,
// centre (2D-3D: its two pixel coordinates), shape (2D-3D) and bound.
__host__ __device__ inline void kp_words(int kind, const float *a, const float *c, const float *L, float beta,
                                         uint32_t w[11]) {
  const bool is2d = kind == PURSE_KIND_2D3D;
  for (int r = 0; r < 3; ++r) w[r] = fbits(a[r]);
  for (int r = 0; r < 3; ++r) w[3 + r] = (r < 2 || !is2d) ? fbits(c[r]) : 0u;
  for (int r = 0; r < 4; ++r) w[6 + r] = is2d ? fbits(L[r]) : 0u;
  w[10] = fbits(beta);
}

// Fingerprint term of the intrinsics (2D-3D), keyed as keypoint -1.
__host__ __device__ inline unsigned long long intrinsics_term(const float K[4]) {
  uint32_t w[11] = {fbits(K[0]), fbits(K[1]), fbits(K[2]), fbits(K[3]), 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  return kp_data_term(-1, w);
}

// Term of the descent signature for step i (i = 0: the first feasible
// sample, the descent's start) whose winner is sample id with rotation
// entries R (the bits of its 9 floats): the iterates are a function of the
// start's and the winners' rotations only, so the signature ties stored
// iterates to exactly the data they were computed from.
__host__ __device__ inline unsigned long long step_sig_term(int i, int id, const uint32_t R[9]) {
  unsigned long long z = trace_mix(i, id);
  for (int k = 0; k < 9; ++k) z = mix64(z ^ ((unsigned long long)R[k] << (k & 1 ? 32 : 0)));
  return z;
}

// Position of s in the sorted active set act[0..n), or -1.
__host__ __device__ inline int find_sorted(const int *act, int n, int s) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    if (act[mid] == s) return mid;
    if (act[mid] < s)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// Inserts sample s into the sorted active set act[0..n) of capacity cap.
// Returns kBwdOk (inserted or already present), kBwdBadTrace when s is not
// a sample id of an instance of M samples (the radius search's sentinel
// INT32_MAX among them), or kBwdOverflow when the set is full.
__host__ __device__ inline int32_t active_insert(int *act, int &n, int cap, int s, int64_t M) {
  if (s < 0 || (int64_t)s >= M) return kBwdBadTrace;
  if (find_sorted(act, n, s) >= 0) return kBwdOk;
  if (n >= cap) return kBwdOverflow;
  int k = n++;
  while (k > 0 && act[k - 1] > s) {
    act[k] = act[k - 1];
    --k;
  }
  act[k] = s;
  return kBwdOk;
}

// One candidate of the radius argmax: a strictly larger distance replaces
// the best (candidates arrive in increasing id per thread).  A NaN distance
// never replaces it, so with a non-finite centre the id stays at the
// sentinel INT32_MAX, which radius_sample_status turns into an error.
__host__ __device__ inline void radius_take(double f, int s, double &best, int &id) {
  if (f > best) {
    best = f;
    id = s;
  }
}

// Merge of two partial radius argmaxes: the larger distance, ties to the
// lower id.
__host__ __device__ inline void radius_merge(double f2, int s2, double &best, int &id) {
  if (f2 > best || (f2 == best && s2 < id)) {
    best = f2;
    id = s2;
  }
}

// The radius sample id found by the search: kBwdOk when it is a sample of
// the instance, kBwdNonFinite otherwise (no finite distance was seen).
__host__ __device__ inline int32_t radius_sample_status(int id, int64_t M) {
  return (id >= 0 && (int64_t)id < M) ? kBwdOk : kBwdNonFinite;
}

// Index of checkpoint q of instance j in the [n_inst][ckpt_count(T, ck)]
// array, or -1 when q is out of range.
__host__ __device__ inline int64_t ckpt_index(int j, int q, int T, int ck) {
  const int nq = ckpt_count(T, ck);
  if (q < 0 || q >= nq) return -1;
  return (int64_t)j * nq + q;
}

}  // namespace purse
