// Workspace records shared by the host library and the kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/purse.h"

namespace purse {

// Per-keypoint record written by the prologue (48 bytes, read wave-uniformly
// by the sampler).
//   3D-3D: m = a_i - abar (centred model point), c = b_i, w unused.
//   2D-3D: m = Z_i, c = (z_i.x, z_i.y, 0), w = (u00, u01, u11) with
//          [[u00, u01], [0, u11]]^T [[u00, u01], [0, u11]] = Lambda_i.
//   kb = kappa beta_i, kb2 = kb^2, bt = beta_i + tau_abs.
struct KpRec {
  float m[3];
  float c[3];
  float w[3];
  float kb;
  float kb2;
  float bt;
};
static_assert(sizeof(KpRec) == 48, "KpRec layout");

// Per-instance record written by the prologue.
struct InstRec {
  int32_t kind, n_kp, status, has_anchor;
  int64_t kp_off, sample_off, n_samples;
  uint64_t seed;
  float Rc[9], tc[3];   // centre pose x_c
  float oc[3];          // pivot o_c = R_c mean(model) + t_c
  float Ra[9], ta[3];   // feasible anchor
  float abar[3];        // model centroid
  float K[4];           // fx, fy, cx, cy
  unsigned long long data_fp;  // fingerprint of the instance's inputs (inst_data_fp)
};
static_assert(sizeof(InstRec) == 192, "InstRec layout");

// MEGB per-instance scratch.
struct MegbRec {
  int32_t first;          // first feasible instance-local index (INT32_MAX if none)
  int32_t n_rescan[2];    // diagnostics: rescans per chain
  int32_t n_global[2];    // diagnostics: full-scan stages per chain (low 16 bits), global shells rebuilt (high 16)
  int32_t n_piped;        // diagnostics: rotation steps taken in pipelined segments
  unsigned long long n_feasible;
  unsigned long long max_rot;    // float64 bit pattern of max ||R* - R_s||_F^2
  unsigned long long max_trans;  // float64 bit pattern of max ||t* - t_s||^2
  float centre[12];       // R* row-major, t*
  long long n_groups[2];  // diagnostics: chunk groups scanned in shell steps per chain
  float4 early_c[2];      // centre after the steps taken by the multi-workgroup first phase
  // global shell of each chain (instances of the first phase): the gs_n
  // samples at distance >= gs_theta from early_c (gs_theta = -1: every
  // feasible sample; gs_n = -1: no shell)
  int32_t gs_n[2];
  float gs_theta[2];
  // rotation iterates C_0, C_ck, C_2ck, ... left for the backward, valid for
  // the trace whose signature is ck_hash (ck_T = 0: none)
  unsigned long long ck_hash;
  int32_t ck_T, ck_every;
  int32_t chain_us[2];    // diagnostics: each chain's workgroup time (device real-time clock, us)
  int32_t n_pipe_fail;    // diagnostics: rotation pipelined segments ended by a failed prediction
  int32_t n_pipe_seg;     // diagnostics: rotation pipelined segments
};
static_assert(sizeof(MegbRec) == 192, "MegbRec layout");

// Instances of at least kBigInstance samples take the first kEarlySteps
// descent steps in kEarlyWG workgroups per chain, one launch per step, and
// then gather their global shell: the farthest samples from the centre the
// first phase reached, at most one in kShellDiv of the instance's samples,
// which the chain's rescans stream instead of every sample.
constexpr int64_t kBigInstance = 32768;
constexpr int kEarlySteps = 32;
constexpr int kEarlyWG = 64;
constexpr int kShellBins = 256;
constexpr int kShellDiv = 16;

// Global-shell slots of an instance: [off / kShellDiv, off / kShellDiv +
// M / kShellDiv) in each chain's array (disjoint between instances, since
// floor(a) + floor(b) <= floor(a + b)).
__host__ __device__ inline int64_t gshell_stride(int64_t total_samples, int64_t max_samples) {
  return max_samples >= kBigInstance ? total_samples / kShellDiv + 1 : 0;
}

// Per-step term of the signature that ties the stored iterates to the
// rotation argmax trace they belong to: the splitmix64 finaliser of (i, id),
// summed over the steps (wrapping), so the sum does not depend on order.
__host__ __device__ inline unsigned long long trace_mix(int i, int id) {
  unsigned long long z = ((unsigned long long)(unsigned)i << 32) | (unsigned)id;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Checkpoint spacing of the rotation iterates and their count per instance.
constexpr int kMaxCkpt = 16;  // largest checkpoint spacing
__host__ __device__ inline int ckpt_spacing(int ckpt_every) {
  return ckpt_every < kMaxCkpt ? (ckpt_every > 0 ? ckpt_every : 1) : kMaxCkpt;
}
__host__ __device__ inline int ckpt_count(int T, int ck) { return (T + ck - 1) / ck; }

// Backward scratch.
constexpr int kMaxActive = 256;  // distinct samples the descent may touch per instance
constexpr int kMaxDirs = 6 * PURSE_MAX_KP;

struct BwdRec {
  int32_t n_act;   // active samples (sorted ids in `active`)
  int32_t status;  // 0 ok, 1 empty, 2 active set beyond capacity, 3 trace inconsistent with mask,
                   // 4 records of another batch or data, 5 non-finite centre
  int32_t s0, sD, sd;
  int32_t n_distinct;  // distinct samples the descent touched (also beyond capacity)
  int32_t active[kMaxActive];
  double cot[kMaxActive][12];  // cotangent of each active pose: R (row-major), t
};

constexpr size_t kAlign = 256;
__host__ __device__ constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct WsLayout {
  size_t inst, kp, sched, megb, quat, trans, dref, bwd, ckpt, tan, contrib, items, early, gid, gpt, total;
};

// First-phase scratch per (instance, chain): the packed (key, ~id) argmax of
// every workgroup for two consecutive steps, the centre for two consecutive
// steps, every workgroup's largest distance, the global shell's histogram
// and its fill count.
struct EarlyScratch {
  unsigned long long part[2][kEarlyWG];
  float4 cbuf[2];
  float dmax[kEarlyWG];
  unsigned int hist[kShellBins];
  int32_t count;
  int32_t pad[3];
};

// Tile schedule of the sampler, one per launch group (3D-3D; 2D-3D with the
// general keypoint loop; 2D-3D with the unrolled one): order[n] lists the
// instances (heaviest per trajectory first), tstart[n + 1] the first tile of
// each entry of that order and, last, the group's tile count.
constexpr int kSchedGroups = 3;
__host__ __device__ inline size_t sched_ints(int64_t n_inst) { return 2 * (size_t)n_inst + 1; }

// Byte offsets of the workspace regions.
inline WsLayout ws_layout(int64_t n_inst, int64_t total_kp, int64_t total_samples, int64_t max_samples, int max_kp,
                          int megb_iters, int ckpt_every) {
  WsLayout L;
  size_t o = 0;
  L.inst = o;
  o += align_up(sizeof(InstRec) * (size_t)n_inst);
  L.kp = o;
  o += align_up(sizeof(KpRec) * (size_t)total_kp);
  L.sched = o;
  o += align_up(sizeof(int32_t) * kSchedGroups * (sched_ints(n_inst) + 1));  // schedules, then queue counters
  L.megb = o;
  o += align_up(sizeof(MegbRec) * (size_t)n_inst);
  L.quat = o;
  o += align_up(16 * (size_t)total_samples);
  L.trans = o;
  o += align_up(16 * (size_t)total_samples);
  L.dref = o;
  o += align_up(8 * (size_t)total_samples);  // one float per sample per chain
  L.bwd = o;
  o += align_up(sizeof(BwdRec) * (size_t)n_inst);
  const int ck = ckpt_spacing(ckpt_every);
  L.ckpt = o;  // rotation checkpoints, [n_inst][ckpt_count] quaternions
  o += align_up(16 * (size_t)n_inst * (size_t)ckpt_count(megb_iters, ck));
  const size_t dirs = 6 * (size_t)max_kp;
  L.tan = o;
  o += align_up(sizeof(float) * 27 * (size_t)n_inst * dirs);
  L.contrib = o;
  o += align_up(sizeof(float) * (size_t)n_inst * kMaxActive * dirs);
  L.items = o;  // work-item prefix sums of the tangent kernels, 2D-3D then 3D-3D
  o += align_up(sizeof(int64_t) * 2 * ((size_t)n_inst + 1));
  const bool big = max_samples >= kBigInstance;
  L.early = o;  // [n_inst][2] first-phase scratch
  o += big ? align_up(sizeof(EarlyScratch) * 2 * (size_t)n_inst) : 0;
  const size_t gs = (size_t)gshell_stride(total_samples, max_samples);
  L.gid = o;  // [2][stride] sample ids of the global shells
  o += align_up(sizeof(int32_t) * 2 * gs);
  L.gpt = o;  // [2][stride] their points (quaternion or translation)
  o += align_up(16 * 2 * gs);
  L.total = o;
  return L;
}

// Instance-local sample range [off, off + M) clipped to a valid range of the
// batch (an inconsistent prefix array yields M = 0).
__host__ __device__ inline void sample_range(const int64_t *sample_off, int j, int64_t total, int64_t max_m,
                                             int64_t &off, int64_t &M) {
  off = sample_off[j];
  M = sample_off[j + 1] - off;
  if (off < 0 || M < 0 || M > max_m || off + M > total) {
    off = 0;
    M = 0;
  }
}

// Kernel-side view of the batch (device pointers + host scalars).
struct DevBatch {
  int32_t n_inst;
  int32_t max_kp;
  int64_t total_kp;
  int64_t total_samples;
  int64_t max_samples;
  const int32_t *kind;
  const int32_t *n_kp;
  const int64_t *kp_off;
  const int64_t *sample_off;
  const float *model_pts;
  const float *centres;
  const float *shapes;
  const float *bounds;
  const float *intrinsics;
  const uint64_t *seed;
};

// Strategic random walk parameters (purse_walk_params as the kernels see it).
constexpr int kWalkMaxPerturb = 256;  // N_P
constexpr int kWalkMaxKeep = 16;      // N_P*
constexpr int kWalkMaxScales = 32;    // N_T
struct WalkParams {
  int32_t n_walks, n_iters, n_perturb, n_keep, n_scales;
  float gamma, omega0, v0, t_pert, r_pert;
};

struct DevParams {
  int32_t n_iters, n_gn, n_bis, megb_iters, megb_avg, centre_gn, ckpt_every, flags;
  float omega0, v0, kappa, tau3, tau2, z_min;
};

}  // namespace purse
