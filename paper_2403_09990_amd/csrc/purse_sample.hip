// The sampler: one trajectory per lane.  Workgroup (tile, instance) covers
// samples [tile * blockDim, (tile + 1) * blockDim) of one instance, so every
// wave reads the same keypoint records (wave-uniform loads) and runs one code
// path; one launch per kind keeps each kind's register allocation separate.
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

template <int KIND>
__global__ void __launch_bounds__(256) k_sample(const InstRec *__restrict__ inst, const KpRec *__restrict__ kprec,
                                                DevParams p, float *__restrict__ poses, uint8_t *__restrict__ mask) {
  const int j = blockIdx.y;
  const InstRec I = inst[j];
  if (I.kind != KIND) return;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= I.n_samples) return;
  const int64_t g = I.sample_off + s;
  float4 *out = reinterpret_cast<float4 *>(poses + 12 * g);
  if ((I.status & 0xFF) != PURSE_INST_OK) {
    out[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    mask[g] = 0;
    return;
  }
  const FrameT<float> F = frame_of<float>(I);
  const KpPlain kpl{kprec + I.kp_off};
  Pose x = initial_pose(F, I.seed, (uint64_t)s, p);
  int n_fb = 0;
  uint8_t m = run_trajectory<KIND>(I, F, kpl, x, p, true, n_fb);
  out[0] = make_float4(x.R[0], x.R[1], x.R[2], x.R[3]);
  out[1] = make_float4(x.R[4], x.R[5], x.R[6], x.R[7]);
  out[2] = make_float4(x.R[8], x.t[0], x.t[1], x.t[2]);
  mask[g] = m;
}

void launch_sample(const DevBatch &b, const DevParams &p, const InstRec *inst, const KpRec *kp, float *poses,
                   uint8_t *mask, int tile, int64_t max_samples, hipStream_t stream) {
  dim3 grid((unsigned)((max_samples + tile - 1) / tile), (unsigned)b.n_inst);
  hipLaunchKernelGGL(k_sample<PURSE_KIND_2D3D>, grid, dim3(tile), 0, stream, inst, kp, p, poses, mask);
  hipLaunchKernelGGL(k_sample<PURSE_KIND_3D3D>, grid, dim3(tile), 0, stream, inst, kp, p, poses, mask);
}

}  // namespace purse
