// Host-side launchers of the kernels (one per translation unit).
#pragma once

#include <hip/hip_runtime.h>

#include "purse_layout.hpp"

namespace purse {

void launch_prologue(const DevBatch &b, const DevParams &p, InstRec *inst, KpRec *kp, int32_t *inst_status,
                     hipStream_t stream);

// Workgroups of one sampler launch (an upper bound on sum_j ceil(M_j / tile)).
int64_t sample_grid(int64_t total_samples, int n_inst, int tile);

// Builds the tile schedule (sched: sched_ints(n_inst) int32 per kind, then
// one work-queue counter per kind) and runs both kinds' trajectories; tile:
// samples per workgroup (64, 128 or 256); waves_per_simd: residency cap (0:
// none).  The launch groups run on the stream and two auxiliary streams
// unless PURSE_FLAG_SERIAL_GROUPS; returns an error (after launching the
// work) if the auxiliary streams' join could not be recorded; launch errors
// are left to hipGetLastError.
hipError_t launch_sample(const DevBatch &b, const DevParams &p, const InstRec *inst, const KpRec *kp,
                         int32_t *sched, float *poses, uint8_t *mask, int tile, int64_t grid_samples,
                         int waves_per_simd, hipStream_t stream);

// ckpt: the rotation iterates C_0, C_ck, ... of every descent, left for the
// backward ([n_inst][ckpt_count] quaternions) with their trace signature in rec.
// es, gid, gpt: the first-phase scratch and the global shells (WsLayout
// early, gid, gpt).
void launch_megb(const DevBatch &b, const DevParams &p, const float *poses, const uint8_t *mask,
                 MegbRec *rec, float4 *quat, float4 *trans, float *dref, float4 *ckpt, EarlyScratch *es,
                 int32_t *gid, float4 *gpt, float *centre, double *radii, int64_t *n_feasible, int32_t *trace,
                 int32_t *inst_status, int64_t max_samples, int64_t total_samples, hipStream_t stream);

// megb / ckpt: the records and checkpoints purse_megb left in the workspace,
// used when the signature matches the given trace; otherwise the descent is
// replayed from the trace and the checkpoints (and signature) rewritten.
// Returns an error (after launching part of the work) if the auxiliary
// stream's join could not be recorded; launch errors are left to hipGetLastError.
hipError_t launch_backward(const DevBatch &b, const DevParams &p, const float *poses, const uint8_t *mask,
                           const int32_t *trace, const double *g_radii, const float *g_centre, const InstRec *inst,
                           const KpRec *kp, MegbRec *megb, BwdRec *recs, float4 *ckpt, float *tan, float *contrib,
                           int64_t *items, float *g_centres, float *g_shapes, float *g_bounds, int32_t *bwd_status,
                           hipStream_t stream);

// The strategic random walks of every start, rotation mode then translation
// mode; centre: [n_inst][12] scratch for the average pose of each instance's
// starts; decisions may be NULL.
void launch_walk(const DevBatch &b, const DevParams &p, const WalkParams &wp, const int64_t *start_off,
                 int64_t total_starts, const float *starts, float *centre, float *poses, uint8_t *mask,
                 int32_t *decisions, hipStream_t stream);

// Step I candidates: one trial per sample slot of the batch.
void launch_init(const DevBatch &b, const DevParams &p, float *poses, uint8_t *mask, hipStream_t stream);

}  // namespace purse
