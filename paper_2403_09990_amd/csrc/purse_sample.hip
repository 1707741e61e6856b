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
#include <algorithm>
#include <mutex>

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
  // the work-queue counters of the three groups
  if (tid < kSchedGroups) sched[(size_t)kSchedGroups * sched_ints(n) + tid] = 0;
}

// The tile of schedule entry b: the entry k of the order with
// tstart[k] <= b < tstart[k + 1].
__device__ __forceinline__ int tile_entry(const int32_t *__restrict__ tstart, int n_inst, int b) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tstart[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <int KIND, int NMAX>
__device__ __forceinline__ void sample_tile(int b, const InstRec *__restrict__ inst, const KpRec *__restrict__ kprec,
                                            const int32_t *__restrict__ order, const int32_t *__restrict__ tstart,
                                            int n_inst, const DevParams &p, float *__restrict__ poses,
                                            uint8_t *__restrict__ mask) {
  const int lo = tile_entry(tstart, n_inst, b);
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

// Work-queue mode: each workgroup takes the next tile of the group's
// schedule from the counter k_schedule cleared, until none is left (every
// workgroup reaches the end of the schedule and leaves).
template <typename F>
__device__ __forceinline__ void tile_queue(int32_t *counter, int total, F &&run) {
  __shared__ int sh_b;
  for (;;) {
    if (threadIdx.x == 0) sh_b = atomicAdd(counter, 1);
    __syncthreads();
    const int b = sh_b;
    __syncthreads();  // (sh_b is read before the next tile's atomic overwrites it)
    if (b >= total) break;
    run(b);
  }
}

template <int KIND, int NMAX, bool QUEUE>
__global__ void __launch_bounds__(256) k_sample(const InstRec *__restrict__ inst, const KpRec *__restrict__ kprec,
                                                int32_t *__restrict__ sched, int n_inst, DevParams p,
                                                float *__restrict__ poses, uint8_t *__restrict__ mask) {
  constexpr int grp = group_of<KIND, NMAX>();
  const int32_t *order = sched + (size_t)grp * sched_ints(n_inst);
  const int32_t *tstart = order + n_inst;
  const int total = tstart[n_inst];
  if (QUEUE) {
    tile_queue(sched + (size_t)kSchedGroups * sched_ints(n_inst) + grp, total,
               [&](int b) { sample_tile<KIND, NMAX>(b, inst, kprec, order, tstart, n_inst, p, poses, mask); });
  } else if ((int)blockIdx.x < total) {
    sample_tile<KIND, NMAX>(blockIdx.x, inst, kprec, order, tstart, n_inst, p, poses, mask);
  }
}

// Lane-group modes of the unrolled 2D-3D group (PURSE_FLAG_PAIR_LANES: G = 2,
// PURSE_FLAG_QUAD_LANES: G = 4): a workgroup of blockDim lanes runs blockDim / G
// trajectories, G lanes each; the instance's keypoint records are staged in
// LDS first.
template <int NMAX, int G>
__device__ __forceinline__ void sample_tile_lanes(int b, KpRec *kp_s, const InstRec *__restrict__ inst,
                                                  const KpRec *__restrict__ kprec, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ tstart, int n_inst, const DevParams &p,
                                                  float *__restrict__ poses, uint8_t *__restrict__ mask) {
  const int lo = tile_entry(tstart, n_inst, b);
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

template <int NMAX, int G, bool QUEUE>
__global__ void __launch_bounds__(256, G == 4 ? 4 : 1) k_sample2d_lanes(const InstRec *__restrict__ inst,
                                                        const KpRec *__restrict__ kprec,
                                                        int32_t *__restrict__ sched, int n_inst, DevParams p,
                                                        float *__restrict__ poses, uint8_t *__restrict__ mask) {
  __shared__ KpRec kp_s[NMAX];
  const int32_t *order = sched + (size_t)2 * sched_ints(n_inst);
  const int32_t *tstart = order + n_inst;
  const int total = tstart[n_inst];
  if (QUEUE) {
    // (the queue's barriers also keep a tile's keypoint records until every
    // lane is done with them)
    tile_queue(sched + (size_t)kSchedGroups * sched_ints(n_inst) + 2, total, [&](int b) {
      sample_tile_lanes<NMAX, G>(b, kp_s, inst, kprec, order, tstart, n_inst, p, poses, mask);
    });
  } else if ((int)blockIdx.x < total) {
    sample_tile_lanes<NMAX, G>(blockIdx.x, kp_s, inst, kprec, order, tstart, n_inst, p, poses, mask);
  }
}

int64_t sample_grid(int64_t total_samples, int n_inst, int tile) {
  // sum_j ceil(M_j / tile) <= total / tile + n_inst
  return total_samples / tile + n_inst;
}

namespace {

// Two auxiliary streams (default priority) and three events per device for
// the concurrent launch groups, created on first use and kept until the
// process ends.
struct GroupAux {
  hipStream_t s[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
  bool ok = false, tried = false;
};
std::mutex g_group_mu;
GroupAux g_group[64];

GroupAux *group_aux() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  GroupAux &a = g_group[dev];
  if (!a.tried) {
    a.tried = true;
    bool ok = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
      ok = hipStreamCreateWithFlags(&a.s[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&a.join[k], hipEventDisableTiming) == hipSuccess;
    a.ok = ok;
  }
  return a.ok ? &a : nullptr;
}

}  // namespace

hipError_t launch_sample(const DevBatch &b, const DevParams &p, const InstRec *inst, const KpRec *kp,
                         int32_t *sched, float *poses, uint8_t *mask, int tile, int64_t grid_samples,
                         int waves_per_simd, hipStream_t stream) {
  hipLaunchKernelGGL(k_schedule, dim3(1), dim3(kSchedBlock), 0, stream, inst, b.n_inst, tile, p.flags, sched);
  // The three launch groups write disjoint samples and read only the
  // prologue's records and the schedules: they run concurrently on the
  // caller's stream and two auxiliary streams (a fork and a join by events,
  // which graph capture records as edges), so one group's tail overlaps the
  // others' work.  Serially on the caller's stream when asked or when the
  // auxiliary streams could not be created or forked to.
  std::unique_lock<std::mutex> lk(g_group_mu);
  GroupAux *aux = (p.flags & PURSE_FLAG_SERIAL_GROUPS) ? nullptr : group_aux();
  hipStream_t gs[3] = {stream, stream, stream};
  if (aux && hipEventRecord(aux->fork, stream) == hipSuccess &&
      hipStreamWaitEvent(aux->s[0], aux->fork, 0) == hipSuccess &&
      hipStreamWaitEvent(aux->s[1], aux->fork, 0) == hipSuccess) {
    gs[1] = aux->s[0];
    gs[2] = aux->s[1];
  } else {
    aux = nullptr;
  }
  // waves per SIMD: at most 8 resident (the hardware's limit), or the cap,
  // which each workgroup's LDS padding enforces: just over the share of the
  // compute unit's LDS that would admit one more workgroup, within the
  // per-workgroup limit less room for the kernels' own LDS (under 1 KB).  The
  // allocation granularity can leave one workgroup fewer than the cap.
  const int wg_waves = tile / 64;
  const int cap = waves_per_simd > 0 ? waves_per_simd : 8;
  const int wg_per_cu = std::max(1, (4 * cap + wg_waves - 1) / wg_waves);
  int dev = 0, n_cu = 256, lds_cu = 163840, lds_block = 65536;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    n_cu = 256;
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
      lds_cu <= 0)
    lds_cu = 163840;
  if (hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      lds_block <= 0)
    lds_block = 65536;
  const size_t lds = waves_per_simd > 0 ? (size_t)std::max(0, std::min(lds_cu / (wg_per_cu + 1) + 512, lds_block - 2048))
                                        : 0;
  const bool queue = (p.flags & PURSE_FLAG_WORK_QUEUE) != 0;
  auto grid_of = [&](int t) {
    const int64_t g = sample_grid(grid_samples, b.n_inst, t);
    return dim3((unsigned)(queue ? std::min<int64_t>(g, (int64_t)n_cu * wg_per_cu) : g));
  };
  const dim3 grid = grid_of(tile);
  if (p.flags & PURSE_FLAG_QUAD_LANES) {
    if (queue)
      hipLaunchKernelGGL((k_sample2d_lanes<kSmallN, 4, true>), grid_of(tile / 4), dim3(tile), lds, stream, inst, kp,
                         sched, b.n_inst, p, poses, mask);
    else
      hipLaunchKernelGGL((k_sample2d_lanes<kSmallN, 4, false>), grid_of(tile / 4), dim3(tile), lds, stream, inst, kp,
                         sched, b.n_inst, p, poses, mask);
  } else if (p.flags & PURSE_FLAG_PAIR_LANES) {
    if (queue)
      hipLaunchKernelGGL((k_sample2d_lanes<kSmallN, 2, true>), grid_of(tile / 2), dim3(tile), lds, stream, inst, kp,
                         sched, b.n_inst, p, poses, mask);
    else
      hipLaunchKernelGGL((k_sample2d_lanes<kSmallN, 2, false>), grid_of(tile / 2), dim3(tile), lds, stream, inst, kp,
                         sched, b.n_inst, p, poses, mask);
  } else if (queue) {
    hipLaunchKernelGGL((k_sample<PURSE_KIND_2D3D, kSmallN, true>), grid, dim3(tile), lds, stream, inst, kp, sched,
                       b.n_inst, p, poses, mask);
  } else {
    hipLaunchKernelGGL((k_sample<PURSE_KIND_2D3D, kSmallN, false>), grid, dim3(tile), lds, stream, inst, kp, sched,
                       b.n_inst, p, poses, mask);
  }
  if (queue) {
    hipLaunchKernelGGL((k_sample<PURSE_KIND_2D3D, 0, true>), grid, dim3(tile), lds, gs[1], inst, kp, sched, b.n_inst,
                       p, poses, mask);
    hipLaunchKernelGGL((k_sample<PURSE_KIND_3D3D, 0, true>), grid, dim3(tile), lds, gs[2], inst, kp, sched, b.n_inst,
                       p, poses, mask);
  } else {
    hipLaunchKernelGGL((k_sample<PURSE_KIND_2D3D, 0, false>), grid, dim3(tile), lds, gs[1], inst, kp, sched,
                       b.n_inst, p, poses, mask);
    hipLaunchKernelGGL((k_sample<PURSE_KIND_3D3D, 0, false>), grid, dim3(tile), lds, gs[2], inst, kp, sched,
                       b.n_inst, p, poses, mask);
  }
  if (aux) {
    for (int k = 0; k < 2; ++k) {
      hipError_t e = hipEventRecord(aux->join[k], aux->s[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, aux->join[k], 0);
      if (e != hipSuccess) return e;  // the caller's stream is not joined to that group
    }
  }
  return hipSuccess;
}

}  // namespace purse
