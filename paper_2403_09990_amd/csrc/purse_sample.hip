// The sampler: one trajectory per lane.  A workgroup covers one tile of
// blockDim consecutive samples of one instance, so every wave reads the same
// keypoint records (wave-uniform loads) and runs one code path; one launch
// per kind keeps each kind's register allocation separate.
//
// Tiles of a ragged batch are dealt from a schedule built on the device after
// the prologue: per kind, the instances in decreasing per-trajectory cost (the
// keypoint count orders it within a kind), each contributing ceil(M_j / tile)
// consecutive tiles.  The hardware dispatches workgroups in index order, so the
// heaviest tiles start first and the tail of the launch is made of light ones
// (longest-processing-time-first list scheduling).
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

constexpr int kSmallN = 16;  // keypoint bound of the unrolled 2D-3D variant

constexpr int kSchedBlock = 1024;

// Launch group of an instance: 0 for 3D-3D (an invalid kind goes there too,
// and its flagged outputs are written as zeros), 1 for 2D-3D with the
// general keypoint loop, 2 for 2D-3D instances of at most kSmallN keypoints
// (the unrolled loop, unless the flags ask for the general one).  The group
// depends on the instance alone, so an instance computes bitwise the same
// samples in any batch.
__device__ __forceinline__ int launch_group(const InstRec &I, int flags) {
  if (I.kind != PURSE_KIND_2D3D) return 0;
  return (I.n_kp <= kSmallN && !(flags & PURSE_FLAG_GENERIC_LOOP)) ? 2 : 1;
}

// Lanes per trajectory of launch group 2.
__host__ __device__ inline int group_lanes(int flags) {
  return (flags & PURSE_FLAG_QUAD_LANES) ? 4 : ((flags & PURSE_FLAG_PAIR_LANES) ? 2 : 1);
}

template <int KIND, int NMAX>
constexpr int group_of() {
  return KIND == PURSE_KIND_3D3D ? 0 : (NMAX > 0 ? 2 : 1);
}

constexpr int kMaxSorted = 8192;  // larger batches keep instance order

// Builds both kinds' schedules in one workgroup: rank of instance j = number
// of instances of the kind that come before it (larger keypoint count, or
// equal count and lower index), then a prefix sum of tile counts in rank order.
__global__ void __launch_bounds__(kSchedBlock) k_schedule(const InstRec *__restrict__ inst, int n, int tile_lanes,
                                                          int flags, int32_t *__restrict__ sched) {
  __shared__ int key[kMaxSorted];
  __shared__ int part[kSchedBlock];
  const int tid = threadIdx.x;
  const bool sorted = n <= kMaxSorted && !(flags & PURSE_FLAG_INSTANCE_ORDER);
  for (int kind = 0; kind < kSchedGroups; ++kind) {
    // samples per tile: one per lane, or one per lane group in the lane-group modes
    const int tile = kind == 2 ? tile_lanes / group_lanes(flags) : tile_lanes;
    int32_t *order = sched + (size_t)kind * sched_ints(n);
    int32_t *tstart = order + n;
    if (sorted) {
      for (int j = tid; j < n; j += kSchedBlock) key[j] = launch_group(inst[j], flags) == kind ? inst[j].n_kp : -1;
      __syncthreads();
      for (int j = tid; j < n; j += kSchedBlock) {
        const int kj = key[j];
        int r = 0;
        for (int i = 0; i < n; ++i) {
          const int ki = key[i];
          r += (ki > kj) || (ki == kj && i < j);
        }
        order[r] = j;
      }
    } else {
      for (int j = tid; j < n; j += kSchedBlock) order[j] = j;
    }
    __threadfence_block();
    __syncthreads();
    // tiles per entry of the order, summed over contiguous chunks per thread
    const int per = (n + kSchedBlock - 1) / kSchedBlock;
    const int b0 = tid * per, b1 = min(n, b0 + per);
    int acc = 0;
    for (int k = b0; k < b1; ++k) {
      const InstRec &I = inst[order[k]];
      acc += launch_group(I, flags) == kind ? (int)((I.n_samples + tile - 1) / tile) : 0;
    }
    part[tid] = acc;
    __syncthreads();
    for (int off = 1; off < kSchedBlock; off <<= 1) {
      const int v = tid >= off ? part[tid - off] : 0;
      __syncthreads();
      part[tid] += v;
      __syncthreads();
    }
    int run = tid ? part[tid - 1] : 0;
    for (int k = b0; k < b1; ++k) {
      tstart[k] = run;
      const InstRec &I = inst[order[k]];
      run += launch_group(I, flags) == kind ? (int)((I.n_samples + tile - 1) / tile) : 0;
    }
    if (tid == kSchedBlock - 1) tstart[n] = part[kSchedBlock - 1];
    __syncthreads();
  }
}

template <int KIND, int NMAX>
__global__ void __launch_bounds__(256) k_sample(const InstRec *__restrict__ inst, const KpRec *__restrict__ kprec,
                                                const int32_t *__restrict__ sched, int n_inst, DevParams p,
                                                float *__restrict__ poses, uint8_t *__restrict__ mask) {
  const int32_t *order = sched + (size_t)group_of<KIND, NMAX>() * sched_ints(n_inst);
  const int32_t *tstart = order + n_inst;
  const int b = blockIdx.x;
  if (b >= tstart[n_inst]) return;
  // the entry k of the order with tstart[k] <= b < tstart[k + 1]
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tstart[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int j = order[lo];
  const InstRec &I = inst[j];
  const int64_t s = (int64_t)(b - tstart[lo]) * blockDim.x + threadIdx.x;
  if (launch_group(I, p.flags) != group_of<KIND, NMAX>() || s >= I.n_samples) return;
  const int64_t g = I.sample_off + s;
  float4 *out = reinterpret_cast<float4 *>(poses + 12 * g);
  if ((I.status & 0xFF) != PURSE_INST_OK) {
    out[0] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
    mask[g] = 0;
    return;
  }
  const FrameRef F = frame_ref(I);
  const KpPlain kpl{kprec + I.kp_off};
  Pose x = initial_pose<float>(F, I.seed, (uint64_t)s, p);
  int n_fb = 0;
  uint8_t m = run_trajectory<KIND, NMAX>(I, F, kpl, x, p, true, n_fb);
  out[0] = make_float4(x.R[0], x.R[1], x.R[2], x.R[3]);
  out[1] = make_float4(x.R[4], x.R[5], x.R[6], x.R[7]);
  out[2] = make_float4(x.R[8], x.t[0], x.t[1], x.t[2]);
  mask[g] = m;
}

// Lane-group modes of the unrolled 2D-3D group (PURSE_FLAG_PAIR_LANES: G = 2,
// PURSE_FLAG_QUAD_LANES: G = 4): a workgroup of blockDim lanes runs blockDim / G
// trajectories, G lanes each; the instance's keypoint records are staged in
// LDS first.
template <int NMAX, int G>
__global__ void __launch_bounds__(256, G == 4 ? 4 : 1) k_sample2d_lanes(const InstRec *__restrict__ inst,
                                                        const KpRec *__restrict__ kprec,
                                                        const int32_t *__restrict__ sched, int n_inst, DevParams p,
                                                        float *__restrict__ poses, uint8_t *__restrict__ mask) {
  __shared__ KpRec kp_s[NMAX];
  const int32_t *order = sched + (size_t)2 * sched_ints(n_inst);
  const int32_t *tstart = order + n_inst;
  const int b = blockIdx.x;
  if (b >= tstart[n_inst]) return;
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tstart[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int j = order[lo];
  const InstRec &I = inst[j];
  if (launch_group(I, p.flags) != 2) return;  // (whole workgroup)
  const bool valid = (I.status & 0xFF) == PURSE_INST_OK;
  if (valid && (int)threadIdx.x < I.n_kp) kp_s[threadIdx.x] = kprec[I.kp_off + threadIdx.x];
  __syncthreads();
  const int64_t s = (int64_t)(b - tstart[lo]) * (blockDim.x / G) + (threadIdx.x / G);
  const int q = threadIdx.x % G;
  if (s >= I.n_samples) return;  // the lanes of a group leave together
  const int64_t g = I.sample_off + s;
  float4 *out = reinterpret_cast<float4 *>(poses + 12 * g);
  if (!valid) {
    if (q == 0) {
      out[0] = make_float4(0.f, 0.f, 0.f, 0.f);
      out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
      out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
      mask[g] = 0;
    }
    return;
  }
  const FrameRef F = frame_ref(I);
  Pose x = initial_pose<float>(F, I.seed, (uint64_t)s, p);
  const uint8_t m = run_trajectory_lanes<NMAX, G>(I, F, kp_s, q, x, p);
  if (q == 0) {
    out[0] = make_float4(x.R[0], x.R[1], x.R[2], x.R[3]);
    out[1] = make_float4(x.R[4], x.R[5], x.R[6], x.R[7]);
    out[2] = make_float4(x.R[8], x.t[0], x.t[1], x.t[2]);
    mask[g] = m;
  }
}

int64_t sample_grid(int64_t total_samples, int n_inst, int tile) {
  // sum_j ceil(M_j / tile) <= total / tile + n_inst
  return total_samples / tile + n_inst;
}

void launch_sample(const DevBatch &b, const DevParams &p, const InstRec *inst, const KpRec *kp, int32_t *sched,
                   float *poses, uint8_t *mask, int tile, hipStream_t stream) {
  hipLaunchKernelGGL(k_schedule, dim3(1), dim3(kSchedBlock), 0, stream, inst, b.n_inst, tile, p.flags, sched);
  const dim3 grid((unsigned)sample_grid(b.total_samples, b.n_inst, tile));
  if (p.flags & PURSE_FLAG_QUAD_LANES) {
    const dim3 grid4((unsigned)sample_grid(b.total_samples, b.n_inst, tile / 4));
    hipLaunchKernelGGL((k_sample2d_lanes<kSmallN, 4>), grid4, dim3(tile), 0, stream, inst, kp, sched, b.n_inst, p,
                       poses, mask);
  } else if (p.flags & PURSE_FLAG_PAIR_LANES) {
    const dim3 grid2((unsigned)sample_grid(b.total_samples, b.n_inst, tile / 2));
    hipLaunchKernelGGL((k_sample2d_lanes<kSmallN, 2>), grid2, dim3(tile), 0, stream, inst, kp, sched, b.n_inst, p,
                       poses, mask);
  } else {
    hipLaunchKernelGGL((k_sample<PURSE_KIND_2D3D, kSmallN>), grid, dim3(tile), 0, stream, inst, kp, sched, b.n_inst,
                       p, poses, mask);
  }
  hipLaunchKernelGGL((k_sample<PURSE_KIND_2D3D, 0>), grid, dim3(tile), 0, stream, inst, kp, sched, b.n_inst, p,
                     poses, mask);
  hipLaunchKernelGGL((k_sample<PURSE_KIND_3D3D, 0>), grid, dim3(tile), 0, stream, inst, kp, sched, b.n_inst, p,
                     poses, mask);
}

}  // namespace purse
