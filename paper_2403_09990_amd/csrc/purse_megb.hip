// Minimum enclosing geodesic balls of the feasible samples by geodesic
// gradient descent, one workgroup per (instance, chain): chain 0 is the
// rotation ball (unit quaternions, Frobenius key ||C - R||_F^2 =
// 2 |a - b|^2 |a + b|^2), chain 1 the translation ball.
//
// Each step needs the farthest sample from the current centre.  The chain
// keeps a shell of candidates in LDS: at a rescan with reference centre C_ref
// and radius r_ref it keeps every sample with d(C_ref, s) >= theta (theta from
// a histogram, so the shell fits).  By the triangle inequality a sample
// outside the shell is at most theta + d(C, C_ref) from the current centre C,
// so when the shell's best exceeds that bound (with a rounding slack) the
// shell argmax is the argmax over all samples and the step is exact; when it
// does not, the chain rescans around the current centre.  Steps on the shell
// run in one wavefront with shuffles only, or, once the winners keep coming
// from a few samples, pipelined: one wavefront runs the descent ahead with
// predicted winners and the others check each step's argmax.
#include <float.h>

#include <type_traits>

#include "purse_bwd_check.hpp"
#include "purse_geodesic.hpp"
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kBins = 256;
constexpr int kGlobalSteps = 64;
// samples per thread of the per-sample passes (k_megb_prep, k_megb_radii):
// kPassPer on instances of at least kPassPerMin samples, else one
constexpr int kPassPer = 4;
constexpr int64_t kPassPerMin = 1 << 17;
constexpr int kChainBlock = 512;  // threads of a pipelined chain workgroup (the larger variant)
constexpr int kChainWaves = kChainBlock / 64;
// Variants of the chain workgroup:
//  - kChainWide: eight waves, a shell of 7168 entries and 256 VGPRs (one
//    chain per compute unit);
//  - kChainNarrow: four waves, a shell of 1280 entries and 128 VGPRs, so that
//    four chains share a compute unit (LDS).
constexpr int kChainWide = 1, kChainNarrow = 2;
template <int V>
constexpr int chain_block() { return V == kChainWide ? kChainBlock : 256; }
template <int V>
constexpr int chain_cap() { return V == kChainWide ? 7168 : 1280; }
constexpr int kUnroll = 8;
constexpr int kCap = 7168;
constexpr int kMaxChunks = kCap / 64;
constexpr int kRecentreChunks = 4;  // a step scanning more chunks than this ...
constexpr int kMinShellSteps = 64;   // ... at least this many steps after a rescan triggers a new one
constexpr int kRecentreDiv = 2048;   // (more chunks, up to kRecentreMax, when a rescan streams more
constexpr int kRecentreMax = 32;     //  entries: one chunk per kRecentreDiv of them)
constexpr int kPipeSteps = 64;       // steps per round of a pipelined segment (one per lane)
constexpr int kVerifySkip = 4;       // wave on wave 0's SIMD (waves go round the 4 SIMDs)
constexpr int kPipeMinSeq = 8;       // steps with no new winner before a pipelined segment, doubled after
constexpr int kPipeMaxSeq = 256;     // each failed prediction up to this
static_assert(kCap % 64 == 0, "chunks of 64 tile the shell");

// Chunks a shell step may scan before its stage ends and the chain rescans
// (once kMinShellSteps steps have been taken since the last rescan).  A
// rescan that streams n_src entries costs in proportion to them, so the more
// it streams the more chunks a step may scan first.
__device__ __forceinline__ int recentre_chunks(int n_src) {
  return min(kRecentreMax, max(kRecentreChunks, n_src / kRecentreDiv));
}

__device__ __forceinline__ bool feasible_pt(float4 a, int chain) {
  return chain == 0 ? (a.x >= 0.f) : (a.w != 0.f);
}

// Squared distance: ||R_a - R_b||_F^2 = 2 |a - b|^2 |a + b|^2 for unit
// quaternions a, b (chain 0; both chords are formed directly, so the key stays
// accurate whichever sign b carries); |a - b|^2 for translations (chain 1).
// The sums are written as explicit fused multiply-adds so that every code path
// (shell steps, full scans, the multi-workgroup first phase) rounds a key the
// same way and takes the same argmax decisions.
__device__ __forceinline__ float sqdist(float4 a, float4 b, int chain) {
  if (chain == 0) {
    const float m0 = a.x - b.x, m1 = a.y - b.y, m2 = a.z - b.z, m3 = a.w - b.w;
    const float p0 = a.x + b.x, p1 = a.y + b.y, p2 = a.z + b.z, p3 = a.w + b.w;
    const float x = fmaf(m3, m3, fmaf(m2, m2, fmaf(m1, m1, m0 * m0)));
    const float y = fmaf(p3, p3, fmaf(p2, p2, fmaf(p1, p1, p0 * p0)));
    return (2.f * x) * y;
  }
  const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z;
  return fmaf(d2, d2, fmaf(d1, d1, d0 * d0));
}

// (key desc, id asc) comparison
__device__ __forceinline__ bool better(float k1, int i1, float k2, int i2) {
  return k1 > k2 || (k1 == k2 && i1 < i2);
}

// Wavefront reductions by DPP row permutes: within each row of 16 lanes
// (quad swaps, half-row and row mirrors), then row broadcasts 15 and 31 carry
// the partial results up, so lane 63 ends with the reduction of all 64 lanes.
__device__ __forceinline__ int wave_max_i32(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x140, 0xF, 0xF, false));  // row_mirror
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_min_i32(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0xB1, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x4E, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x141, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x140, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x142, 0xA, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x143, 0xC, 0xF, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// Keys are squared distances (>= 0) or the sentinel -1: their float bit
// patterns order like the values under signed integer comparison.
__device__ __forceinline__ float wave_max_key(float k) { return __int_as_float(wave_max_i32(__float_as_int(k))); }

// Wavefront argmax (key desc, id asc); every lane gets the winning key and id.
__device__ __forceinline__ void wave_argmax(float k, int id, float &wk, int &wi) {
  wk = wave_max_key(k);
  wi = wave_min_i32(k == wk ? id : INT32_MAX);
}

// Running sum of the last iterates: rotation matrices (chain 0) or centres.
// The rotation of the unit quaternion (w, x, y, z) is written out with
// explicit fused multiply-adds, so that every code path (full scans, shell
// steps) rounds the sum the same way.
__device__ __forceinline__ void accumulate_iterate(float4 C, int chain, float acc[9]) {
  if (chain == 0) {
    const float w = C.x, x = C.y, y = C.z, z = C.w;
    acc[0] += fmaf(-2.f, fmaf(y, y, z * z), 1.f);
    acc[1] = fmaf(2.f, fmaf(x, y, -(w * z)), acc[1]);
    acc[2] = fmaf(2.f, fmaf(x, z, w * y), acc[2]);
    acc[3] = fmaf(2.f, fmaf(x, y, w * z), acc[3]);
    acc[4] += fmaf(-2.f, fmaf(x, x, z * z), 1.f);
    acc[5] = fmaf(2.f, fmaf(y, z, -(w * x)), acc[5]);
    acc[6] = fmaf(2.f, fmaf(x, z, -(w * y)), acc[6]);
    acc[7] = fmaf(2.f, fmaf(y, z, w * x), acc[7]);
    acc[8] += fmaf(-2.f, fmaf(x, x, y * y), 1.f);
  } else {
    acc[0] += C.x;
    acc[1] += C.y;
    acc[2] += C.z;
  }
}

__device__ __forceinline__ float wave_max(float v) { return wave_max_key(v); }

// Streams elements [0, M) of src to the workgroup in rounds of
// BLOCK * kUnroll elements (element s0 + u * BLOCK + tid to thread
// tid, past M the pad value).  The loads of the next round are issued before
// the current round is handed to f(vals, s0), so two rounds are in flight.
// Loads are unconditional at an index clamped to M - 1 (vector loads, and no
// branch that would make the wait counts conservative); the pad is selected
// afterwards.
template <int BLOCK, int U = kUnroll, typename T, typename F>
__device__ __forceinline__ void stream_rounds(const T *__restrict__ src, int M, T pad, F &&f) {
  constexpr int R = BLOCK * U;
  if (M <= 0) return;
  const int tid = threadIdx.x;
  const int last = M - 1;
  T cur[U];
#pragma unroll
  for (int u = 0; u < U; ++u) cur[u] = src[min(u * BLOCK + tid, last)];
  for (int s0 = 0; s0 < M; s0 += R) {
    T nxt[U];  // (the last round reloads in-range elements it does not use)
#pragma unroll
    for (int u = 0; u < U; ++u) nxt[u] = src[min(s0 + R + u * BLOCK + tid, last)];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = s0 + u * BLOCK + tid < M ? cur[u] : pad;
    f(v, s0);
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
  }
}

}  // namespace

__global__ void k_megb_init(int n_inst, MegbRec *rec) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_inst) return;
  rec[j].first = INT32_MAX;
  rec[j].n_feasible = 0ull;
  rec[j].max_rot = 0ull;
  rec[j].max_trans = 0ull;
  rec[j].gs_n[0] = rec[j].gs_n[1] = -1;
  rec[j].gs_theta[0] = rec[j].gs_theta[1] = -1.f;
  rec[j].ck_hash = 0ull;
  rec[j].ck_T = 0;
  rec[j].ck_every = 0;
}

// Bin of d among kBins bins of width 1 / rw from lo (rw the reciprocal of
// the width, so a pass over every sample takes no division).  The rounding of
// the product can move d by one bin near an edge, which shifts the bins'
// edges as bounds by about 1e-7 of the distance, far inside the shell
// checks' slack; every pass uses this same function, so counts and members
// agree.
__device__ __forceinline__ int bin_of(float d, float lo, float rw) {
  int b = (int)((d - lo) * rw);
  return b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
}

static_assert(kShellBins == kBins, "one binning for the global and the chain shells");

// The first kEarlySteps steps move the centre across the whole sample cloud,
// so each needs a scan of every feasible sample.  For instances of at least
// kBigInstance samples these scans are spread over kEarlyWG workgroups per
// chain, one launch per step (k_megb_early); smaller instances take them
// inside their chain's workgroup.  Host and device apply the same rule.
constexpr int kEarlyBlock = 256;

__host__ __device__ inline bool early_phase_applies(int64_t M, int T, int avg, int no_prune) {
  return M >= kBigInstance && T > kEarlySteps + avg && !no_prune;
}

// Samples [sb, se) of workgroup b of a chain: kEarlyWG ranges of a multiple
// of kEarlyBlock samples.
__device__ __forceinline__ void early_range(int M, int b, int &sb, int &se) {
  const int span = ((M + kEarlyWG - 1) / kEarlyWG + kEarlyBlock - 1) / kEarlyBlock * kEarlyBlock;
  sb = min(M, b * span);
  se = min(M, sb + span);
}

// Largest 64-bit value of the wavefront (unsigned), in every lane.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}

// (key, id) packed so that an unsigned maximum keeps the larger key and, on
// equal keys, the lower id; keys are >= 0 (a -0 is taken as +0, which it
// equals).  0: no sample.
__device__ __forceinline__ unsigned long long pack_best(float k, int id) {
  return id == INT32_MAX ? 0ull
                         : ((unsigned long long)(__float_as_uint(k) & 0x7fffffffu) << 32) |
                               (unsigned long long)(~(unsigned)id);
}

// Step i of the first phase for every (instance, chain) the rule selects,
// whose feasible samples outnumber the shell capacity (else the shell holds
// them all and the chain's workgroup needs no full scans).  Every workgroup
// first completes step i - 1 itself: it reduces the kEarlyWG packed argmaxes
// the previous launch left and takes the geodesic step from the centre that
// launch started from, so all workgroups hold the same centre with no atomic
// or fence (kernel boundaries order the launches); workgroup 0 records the
// trace, the checkpoint and the centre for the next launch.  Then each
// workgroup finds the farthest of its samples and leaves its packed argmax.
// Launch kEarlySteps + 1 only completes the last step and, as the first pass
// of the global shell, writes every sample's distance from that centre to
// dref and each workgroup's largest distance.  Buffers alternate between
// consecutive launches, so a launch never writes what it reads.
__global__ void __launch_bounds__(kEarlyBlock) k_megb_early(const int64_t *__restrict__ sample_off, int64_t total,
                                                            int64_t max_m, const float4 *__restrict__ quat,
                                                            const float4 *__restrict__ trans, MegbRec *rec,
                                                            EarlyScratch *es, float *dref_all, int32_t *trace,
                                                            float4 *ckpt, int ck, int T, int avg, int cap,
                                                            int no_prune, int i) {
  const int j = blockIdx.z, chain = blockIdx.y, b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t off, M64;
  sample_range(sample_off, j, total, max_m, off, M64);
  if (!early_phase_applies(M64, T, avg, no_prune)) return;
  const int M = (int)M64;  // >= kBigInstance here
  const int first = rec[j].first;
  if (first == INT32_MAX || (int64_t)rec[j].n_feasible <= cap) return;
  const float4 *D = (chain ? trans : quat) + off;
  EarlyScratch &e = es[2 * j + chain];
  int sb, se;
  early_range(M, b, sb, se);
  // ---- the centre before step i (every wave reduces the partials itself)
  float4 C;
  if (i == 1) {
    C = D[first];
  } else {
    static_assert(kEarlyWG == 64, "one partial per lane");
    const unsigned long long best = wave_max_u64(e.part[(i - 1) & 1][lane]);
    const int bi = best ? (int)~(unsigned)(best & 0xffffffffull) : INT32_MAX;
    const float4 Cp = e.cbuf[i & 1];
    C = bi < M ? geodesic_step(Cp, D[bi], i - 1, chain) : Cp;
    if (b == 0 && tid == 0) trace[((int64_t)j * T + i - 2) * 2 + chain] = bi;
  }
  if (b == 0 && tid == 0) {
    e.cbuf[(i + 1) & 1] = C;
    if (i <= kEarlySteps && chain == 0 && (i - 1) % ck == 0) ckpt[(int64_t)j * ckpt_count(T, ck) + (i - 1) / ck] = C;
    if (i > kEarlySteps) rec[j].early_c[chain] = C;
  }
  __shared__ float red_k[kEarlyBlock / 64];
  __shared__ int red_i[kEarlyBlock / 64];
  if (i <= kEarlySteps) {
    // ---- step i over this workgroup's samples
    float bk = -1.f;
    int bi = INT32_MAX;
    stream_rounds<kEarlyBlock>(D + sb, se - sb, make_float4(-2.f, 0.f, 0.f, 0.f), [&](const float4 *a, int s0) {
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int s = sb + s0 + u * kEarlyBlock + tid;
        if (s < se && feasible_pt(a[u], chain)) {
          const float k = sqdist(C, a[u], chain);
          if (better(k, s, bk, bi)) {
            bk = k;
            bi = s;
          }
        }
      }
    });
    float wk;
    int wi;
    wave_argmax(bk, bi, wk, wi);
    if (lane == 0) {
      red_k[wave] = wk;
      red_i[wave] = wi;
    }
    __syncthreads();
    if (tid == 0) {
      bk = red_k[0];
      bi = red_i[0];
#pragma unroll
      for (int w = 1; w < kEarlyBlock / 64; ++w)
        if (better(red_k[w], red_i[w], bk, bi)) {
          bk = red_k[w];
          bi = red_i[w];
        }
      e.part[i & 1][b] = pack_best(bk, bi);
    }
    return;
  }
  // ---- global shell, first pass: distances from the centre
  float *dref = dref_all + chain * total + off;
  float mx = 0.f;
  stream_rounds<kEarlyBlock>(D + sb, se - sb, make_float4(-2.f, 0.f, 0.f, 0.f), [&](const float4 *a, int s0) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int s = sb + s0 + u * kEarlyBlock + tid;
      if (s < se) {
        float d = -1.f;
        if (feasible_pt(a[u], chain)) {
          d = __builtin_amdgcn_sqrtf(sqdist(C, a[u], chain));
          mx = fmaxf(mx, d);
        }
        dref[s] = d;
      }
    }
  });
  mx = wave_max(mx);
  if (lane == 0) red_k[wave] = mx;
  if (b == 0) {
    for (int k = tid; k < kShellBins; k += kEarlyBlock) e.hist[k] = 0u;
    if (tid == 0) e.count = 0;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int w = 1; w < kEarlyBlock / 64; ++w) mx = fmaxf(mx, red_k[w]);
    e.dmax[b] = fmaxf(mx, red_k[0]);
  }
}

// Histogram bin width of a chain's global shell: the largest distance over
// kShellBins (every workgroup computes it the same way); 0 when every
// feasible sample sits at the centre.
__device__ __forceinline__ float gshell_width(const EarlyScratch &e) {
  static_assert(kEarlyWG == 64, "one entry per lane");
  return wave_max(e.dmax[threadIdx.x & 63]) / (float)kShellBins;
}

// Global shell, second pass: histogram of the distances over [0, max].
__global__ void __launch_bounds__(kEarlyBlock) k_megb_gshell_hist(const int64_t *__restrict__ sample_off,
                                                                  int64_t total, int64_t max_m, MegbRec *rec,
                                                                  EarlyScratch *es, const float *dref_all, int T,
                                                                  int avg, int cap, int no_prune) {
  const int j = blockIdx.z, chain = blockIdx.y, b = blockIdx.x;
  const int tid = threadIdx.x;
  int64_t off, M64;
  sample_range(sample_off, j, total, max_m, off, M64);
  if (!early_phase_applies(M64, T, avg, no_prune)) return;
  if (rec[j].first == INT32_MAX || (int64_t)rec[j].n_feasible <= cap) return;
  EarlyScratch &e = es[2 * j + chain];
  const float w = gshell_width(e);
  if (!(w > 0.f)) return;
  const float rw = 1.f / w;
  __shared__ unsigned int h[kShellBins];
  for (int k = tid; k < kShellBins; k += kEarlyBlock) h[k] = 0u;
  __syncthreads();
  int sb, se;
  early_range((int)M64, b, sb, se);
  const float *dref = dref_all + chain * total + off;
  stream_rounds<kEarlyBlock, 16>(dref + sb, se - sb, -1.f, [&](const float *dd, int) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (dd[u] >= 0.f) atomicAdd(&h[bin_of(dd[u], 0.f, rw)], 1u);
  });
  __syncthreads();
  for (int k = tid; k < kShellBins; k += kEarlyBlock)
    if (h[k]) atomicAdd(&e.hist[k], h[k]);
}

// Global shell, third pass: the threshold (the lowest bin edge above which at
// most M / kShellDiv samples lie) and the members, compacted into the
// chain's slots: each workgroup counts its members per wave, reserves its
// range with one atomic, and writes them wave by wave in sample order.  The
// order of the workgroups' ranges varies from run to run; every use of the
// shell is order-independent (argmax ties go to the lowest sample id).
__global__ void __launch_bounds__(kEarlyBlock) k_megb_gshell_collect(const int64_t *__restrict__ sample_off,
                                                                     int64_t total, int64_t max_m,
                                                                     const float4 *__restrict__ quat,
                                                                     const float4 *__restrict__ trans,
                                                                     MegbRec *rec, EarlyScratch *es,
                                                                     const float *dref_all, int32_t *gid_all,
                                                                     float4 *gpt_all, int64_t gstride, int T,
                                                                     int avg, int cap, int no_prune) {
  const int j = blockIdx.z, chain = blockIdx.y, b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t off, M64;
  sample_range(sample_off, j, total, max_m, off, M64);
  if (!early_phase_applies(M64, T, avg, no_prune)) return;
  if (rec[j].first == INT32_MAX || (int64_t)rec[j].n_feasible <= cap) return;
  EarlyScratch &e = es[2 * j + chain];
  const float w = gshell_width(e);
  if (!(w > 0.f)) return;  // no shell (gs_n stays -1)
  const float rw = 1.f / w;
  const int M = (int)M64;
  const int G = M / kShellDiv;
  __shared__ int sh_bstar, sh_n;
  __shared__ int wcount[kEarlyBlock / 64], wbase[kEarlyBlock / 64];
  if (tid == 0) {
    int cum = 0, bb = kShellBins - 1;
    for (; bb >= 0; --bb) {
      if (cum + (int)e.hist[bb] > G) break;
      cum += (int)e.hist[bb];
    }
    // bb < 0: every feasible sample fits; bb = kShellBins - 1: the top bin
    // alone is too large (no shell)
    sh_bstar = bb + 1;
    sh_n = cum;
    if (b == 0) {
      rec[j].gs_n[chain] = bb == kShellBins - 1 ? -1 : cum;
      rec[j].gs_theta[chain] = bb < 0 ? -1.f : (float)(bb + 1) * w;
    }
  }
  __syncthreads();
  const int bstar = sh_bstar;
  if (bstar >= kShellBins) return;
  int sb, se;
  early_range(M, b, sb, se);
  // each wave takes a contiguous quarter of the range
  const int q = ((se - sb + kEarlyBlock / 64 - 1) / (kEarlyBlock / 64) + 63) / 64 * 64;
  const int wb = min(se, sb + wave * q), we = min(se, wb + q);
  const float *dref = dref_all + chain * total + off;
  auto member = [&](float d) { return d >= 0.f && bin_of(d, 0.f, rw) >= bstar; };
  int cnt = 0;
  for (int s = wb + lane; s < we; s += 64) cnt += member(dref[s]) ? 1 : 0;
  for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if (lane == 0) wcount[wave] = cnt;
  __syncthreads();
  if (tid == 0) {
    int t = 0;
    for (int k = 0; k < kEarlyBlock / 64; ++k) {
      wbase[k] = t;
      t += wcount[k];
    }
    const int base = t ? atomicAdd(&e.count, t) : 0;
    for (int k = 0; k < kEarlyBlock / 64; ++k) wbase[k] += base;
  }
  __syncthreads();
  const float4 *D = (chain ? trans : quat) + off;
  int32_t *gid = gid_all + chain * gstride + off / kShellDiv;
  float4 *gpt = gpt_all + chain * gstride + off / kShellDiv;
  int pos = wbase[wave];
  for (int s0 = wb; s0 < we; s0 += 64) {
    const int s = s0 + lane;
    const bool m = s < we && member(dref[s]);
    const unsigned long long mk = __ballot(m);
    const int p = pos + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
    if (m && p < G) {
      gid[p] = s;
      gpt[p] = D[s];
    }
    pos += __popcll(mk);
  }
  (void)sh_n;
}

// Per sample: quaternion (w >= 0; w = -2 marks an infeasible sample) and
// translation (w = 1 feasible, 0 not); first feasible index; feasible count.
template <int PER>
__global__ void __launch_bounds__(kBlock) k_megb_prep(const int64_t *__restrict__ sample_off, int64_t total,
                                                      int64_t max_m, const float *__restrict__ poses,
                                                      const uint8_t *__restrict__ mask, MegbRec *rec,
                                                      float4 *quat, float4 *trans) {
  const int j = blockIdx.y;
  int64_t off, M;
  sample_range(sample_off, j, total, max_m, off, M);
  const int64_t s0 = (int64_t)blockIdx.x * (kBlock * PER) + threadIdx.x;
  __shared__ int cnt[kWaves];
  __shared__ int firsts[kWaves];
  int feas = 0, first = INT32_MAX;
  // PER samples per thread, kBlock apart: the masks first, then the
  // poses of the feasible ones, every load of a round in flight together
  uint8_t m[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t s = s0 + u * kBlock;
    m[u] = s < M ? mask[off + s] : (uint8_t)0;
  }
  float4 a[PER], b[PER], c[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t s = s0 + u * kBlock;
    if (s < M && (m[u] & PURSE_MASK_FEASIBLE)) {
      const float4 *pp = reinterpret_cast<const float4 *>(poses + 12 * (off + s));
      a[u] = pp[0];
      b[u] = pp[1];
      c[u] = pp[2];
    }
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int64_t s = s0 + u * kBlock;
    if (s >= M) continue;
    const int64_t g = off + s;
    if (m[u] & PURSE_MASK_FEASIBLE) {
      float R[9] = {a[u].x, a[u].y, a[u].z, a[u].w, b[u].x, b[u].y, b[u].z, b[u].w, c[u].x};
      quat[g] = quat_from_rot(R);
      trans[g] = make_float4(c[u].y, c[u].z, c[u].w, 1.f);
      ++feas;
      first = min(first, (int)s);
    } else {
      quat[g] = make_float4(-2.f, 0.f, 0.f, 0.f);
      trans[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  // block reduction, one atomic per block
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    feas += __shfl_xor(feas, o, 64);
    first = min(first, __shfl_xor(first, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    cnt[w] = feas;
    firsts[w] = first;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0, f = INT32_MAX;
    for (int k = 0; k < kWaves; ++k) {
      c += cnt[k];
      f = min(f, firsts[k]);
    }
    if (c) {
      atomicAdd(&rec[j].n_feasible, (unsigned long long)c);
      atomicMin(&rec[j].first, f);
    }
  }
}

// A chain's global shell (the state only rescans read) and its diagnostics.
struct ChainGs {
  int n, built_at, n_built;
  float theta;
  float4 C;
};
struct ChainDiag {
  int n_rescan, n_global, n_seg, n_piped, n_fail;
  long long n_groups;
  uint64_t t_start;
};

// Shared state of one chain's workgroup.
struct ChainShared {
  float4 *pt;             // shell points, [cap]
  int *id;                // shell sample ids, [cap]
  unsigned int *hist;     // [kBins]
  unsigned int *cursor;   // [kBins]
  float *chunk_ub;        // [kMaxChunks]
  float (*red_k)[kChainWaves];
  int (*red_i)[kChainWaves];
};

template <int CHAIN, int V>
__device__ __forceinline__ void chain_run(const ChainShared &S, const int64_t *__restrict__ sample_off,
                                          int64_t max_m, const float4 *__restrict__ pts, MegbRec *rec,
                                          float *dref_all, int64_t total_samples, int32_t *trace,
                                          float4 *ckpt_all, int ck, int T, int avg, int cap, int no_prune,
                                          int32_t *__restrict__ gid_all, float4 *__restrict__ gpt_all,
                                          int64_t gstride) {
  __shared__ float4 st_C;
  __shared__ int st_i;
  __shared__ float st_theta, st_lo, st_w, st_rref;
  __shared__ int st_bstar;
  __shared__ int st_mode;  // 0 shell in LDS, 1 scan of every sample
  __shared__ unsigned int sh_n;
  // pipelined shell steps
  __shared__ float4 pl_C[3][kPipeSteps];  // starting iterate of each step of a round (3 rounds in flight)
  __shared__ int pl_W[3][kPipeSteps];     // and its predicted winner
  __shared__ int pl_fail[3];              // first step of a round whose prediction failed
  __shared__ float4 pl_Cend;
  __shared__ int pl_go;

  constexpr int chain = CHAIN;
  constexpr int BLK = chain_block<V>(), NW = BLK / 64;
  // verifier waves of a pipelined segment: every wave but wave 0 and, in the
  // eight-wave group, the one that shares wave 0's SIMD (waves go round the
  // four SIMDs)
  constexpr int kSkipWave = NW > 4 ? kVerifySkip : NW;
  constexpr int kVerifiers = NW > 4 ? NW - 2 : NW - 1;
  // elements per thread and round in the passes over d_ref: the wide variant
  // has the registers to keep more loads in flight, which these
  // latency-bound passes of one workgroup need
  constexpr int UF = V == kChainWide ? 32 : kUnroll;
  const int j = blockIdx.x >> 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t off, M64;
  sample_range(sample_off, j, total_samples, max_m, off, M64);
  const int M = (int)M64;
  const float4 *D = pts + off;
  float *dref = dref_all + chain * total_samples + off;
  int32_t *tr = trace + (int64_t)j * T * 2 + chain;
  // rotation iterates C_{q ck} for the backward (each step's path leaves the
  // ones it starts from)
  float4 *ckq = ckpt_all + (int64_t)j * ckpt_count(T, ck);
  const int first = rec[j].first;
  if (first == INT32_MAX) {
    for (int k = tid; k < T; k += BLK) tr[2 * k] = -1;
    return;
  }
  const int n_feas = (int)rec[j].n_feasible;
  // the first steps were taken by k_megb_early when the rule selects it,
  // which also gathered the global shell: the gs_n samples at distance
  // >= gs_theta from C_g (gs_theta = -1: every feasible sample).  Samples
  // outside it lie within gs_theta + d(C, C_g) of any centre C, so rescans
  // stream the shell alone while that bound stays below the farthest member.
  const bool ep = early_phase_applies(M64, T, avg, no_prune) && n_feas > cap;
  int32_t *gid = gid_all + chain * gstride + off / kShellDiv;
  float4 *gpt = gpt_all + chain * gstride + off / kShellDiv;
  // A global shell that no longer certifies any step (the centre has moved
  // too far from C_g) is rebuilt around the centre of the next full rescan,
  // from the distances that rescan computes, at most once per kMinShellSteps
  // steps.  Its state, which only rescans read, and the diagnostics live in
  // LDS (thread 0 writes them between barriers), so that the stepping loops
  // keep their registers.
  const int gs_cap = M / kShellDiv;
  __shared__ ChainGs sg;
  __shared__ ChainDiag sdg;
  if (tid == 0) {
    st_C = ep ? rec[j].early_c[chain] : D[first];
    st_i = ep ? kEarlySteps + 1 : 1;
    sg.n = ep ? rec[j].gs_n[chain] : -1;
    sg.theta = ep ? rec[j].gs_theta[chain] : -1.f;
    sg.C = rec[j].early_c[chain];
    sg.built_at = ep ? -kMinShellSteps : INT32_MAX;
    sg.n_built = 0;
    sdg = ChainDiag{0, 0, 0, 0, 0, 0ll, __builtin_amdgcn_s_memrealtime()};
  }
  __syncthreads();
  bool use_gs = sg.n > 0;
  float acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.f;
  bool stalled = false;
  int recentre = kRecentreChunks;  // chunks a shell step may scan (set by each rescan)
  int stage_groups = 0;

  while (true) {
    const float4 Cref = st_C;
    const int i0 = st_i;
    if (i0 > T) break;
    const bool early = i0 <= kEarlySteps;
    const bool global = (no_prune || stalled || early) && n_feas > cap;
    if (!global) {
      // -------------------------------------------------------------- rescan
      if (tid == 0) ++sdg.n_rescan;
      // entries: the global shell's or every sample
      const bool from_gs = use_gs;  // (a rebuild below does not change this rescan's source)
      const float4 *src = from_gs ? gpt : D;
      const int n_src = from_gs ? sg.n : M;
      const int n_src_feas = from_gs ? sg.n : n_feas;
      recentre = recentre_chunks(n_src);
      float mx = 0.f;
      stream_rounds<BLK>(src, n_src, make_float4(-2.f, 0.f, 0.f, 0.f), [&](const float4 *a, int s0) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          int s = s0 + u * BLK + tid;
          if (s < n_src) {
            float d = -1.f;
            if (feasible_pt(a[u], chain)) {
              d = __builtin_amdgcn_sqrtf(sqdist(Cref, a[u], chain));  // within the slack
              mx = fmaxf(mx, d);
            }
            dref[s] = d;
          }
        }
      });
      mx = wave_max(mx);
      if (lane == 0) S.red_k[0][wave] = mx;
      __syncthreads();
      float rref = 0.f;
#pragma unroll
      for (int k = 0; k < NW; ++k) rref = fmaxf(rref, S.red_k[0][k]);
      // (the narrow variant, which runs batches of more chains than compute
      // units, keeps its registers for four chains per compute unit and
      // leaves a stale global shell to full rescans)
      if (V == kChainWide && ep && !use_gs && i0 - sg.built_at >= kMinShellSteps) {
        // ---------------------------------- rebuild the global shell at C_ref
        const float gw = rref / (float)kShellBins;
        if (gw > 0.f) {
          const float grw = 1.f / gw;
          for (int k = tid; k < kBins; k += BLK) S.hist[k] = 0u;
          __syncthreads();
          // (a short unroll: the rebuild is rare, and its registers would
          // otherwise be taken from the stepping loops)
          stream_rounds<BLK, kUnroll>(dref, M, -1.f, [&](const float *dd, int) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
              if (dd[u] >= 0.f) atomicAdd(&S.hist[bin_of(dd[u], 0.f, grw)], 1u);
          });
          __syncthreads();
          if (tid == 0) {
            int cum = 0, bb = kShellBins - 1;
            for (; bb >= 0; --bb) {
              if (cum + (int)S.hist[bb] > gs_cap) break;
              cum += (int)S.hist[bb];
            }
            st_bstar = bb == kShellBins - 1 ? -1 : bb + 1;  // -1: the top bin alone is too large
            sh_n = 0u;
            if (st_bstar < 0) sg.n = -1;
          }
          __syncthreads();
          const int gb = st_bstar;
          if (gb >= 0) {
            stream_rounds<BLK, kUnroll>(dref, M, -1.f, [&](const float *dd, int s0) {
#pragma unroll
              for (int u = 0; u < kUnroll; ++u) {
                const int s = s0 + u * BLK + tid;
                if (dd[u] >= 0.f && bin_of(dd[u], 0.f, grw) >= gb) {
                  const unsigned int pos = atomicAdd(&sh_n, 1u);
                  if (pos < (unsigned)gs_cap) {
                    gid[pos] = s;
                    gpt[pos] = D[s];
                  }
                }
              }
            });
            __syncthreads();
            if (tid == 0) {
              sg.n = min((int)sh_n, gs_cap);
              sg.theta = gb == 0 ? -1.f : (float)gb * gw;
              sg.C = Cref;
              ++sg.n_built;
            }
          }
        }
        if (tid == 0) sg.built_at = i0;
        __syncthreads();
        use_gs = sg.n > 0;
      }
      // bound of every sample outside the global shell
      float theta_out = -1.f;
      if (from_gs && sg.theta >= 0.f) {
        theta_out = sg.theta + __builtin_amdgcn_sqrtf(sqdist(Cref, sg.C, chain));
        if (!(theta_out < rref)) {
          // the shell can no longer certify a step: rescan every sample
          use_gs = false;
          __syncthreads();  // (S.red_k is read above and written by the next rescan)
          continue;
        }
      }
      // Shell membership: d >= theta and (coarse) bin >= bstar of the
      // histogram (lo, w); theta = -1 when every feasible sample fits.  The
      // global shell's entries lie at least gs_theta - d(C_ref, C_g) from
      // C_ref, so its histogram starts there (spread over all the bins, not
      // piled into the top few); an entry rounded below lo is within
      // theta_out, which the stage's bound includes.
      if (tid == 0) {
        const float lo0 = from_gs && theta_out >= 0.f ? fmaxf(0.f, 2.f * sg.theta - theta_out - 1e-5f * rref) : 0.f;
        st_mode = 0;
        st_theta = -1.f;
        st_lo = lo0;
        st_w = (rref - lo0) / (float)kBins;
        st_bstar = 0;
        st_rref = rref;
      }
      __syncthreads();
      if (n_src_feas > cap) {
        for (int level = 0; level < 2; ++level) {
          const float lo = st_lo, wdt = st_w;
          if (!(wdt > 0.f)) {
            if (tid == 0) st_mode = 1;
            __syncthreads();
            break;
          }
          for (int k = tid; k < kBins; k += BLK) S.hist[k] = 0u;
          __syncthreads();
          const float rw = 1.f / wdt;
          stream_rounds<BLK, UF>(dref, n_src, -1.f, [&](const float *dd, int) {
#pragma unroll
            for (int u = 0; u < UF; ++u)
              if (dd[u] >= lo && dd[u] >= 0.f) atomicAdd(&S.hist[bin_of(dd[u], lo, rw)], 1u);
          });
          __syncthreads();
          if (tid == 0) {
            int cum = 0, bb = kBins - 1;
            for (; bb >= 0; --bb) {
              if (cum + (int)S.hist[bb] > cap) break;
              cum += (int)S.hist[bb];
            }
            if (bb < 0) {  // everything at or above lo fits
              st_bstar = 0;
              st_theta = level == 0 ? -1.f : lo;
            } else if (bb < kBins - 1) {
              st_bstar = bb + 1;
              st_theta = lo + (float)(bb + 1) * wdt;
            } else if (level == 0) {  // the top bin alone overflows: refine inside it
              st_lo = lo + (float)(kBins - 1) * wdt;
              st_w = wdt / (float)kBins;
              st_theta = -2.f;
            } else {
              st_mode = 1;
            }
          }
          __syncthreads();
          if (st_theta != -2.f || st_mode == 1) break;
        }
      }
      // samples outside the global shell are bounded by theta_out
      if (from_gs && tid == 0 && st_mode == 0) st_theta = fmaxf(st_theta, theta_out);
      __syncthreads();
      // ---------------- collect, ordered by fine bins over [max(theta,0), rref]
      if (st_mode == 0) {
        const float lo = st_lo, wdt = st_w, theta = st_theta;
        const int bstar = st_bstar;
        const float flo = fmaxf(theta, 0.f);
        const float fw = (rref - flo) / (float)kBins;
        const bool fine = fw > 0.f;
        const float rw = wdt > 0.f ? 1.f / wdt : 0.f, rfw = fine ? 1.f / fw : 0.f;
        auto member = [&](float d) {
          return d >= 0.f && d >= theta && (theta < 0.f || (d >= lo && bin_of(d, lo, rw) >= bstar));
        };
        auto fbin = [&](float d) { return fine ? bin_of(d, flo, rfw) : kBins - 1; };
        for (int k = tid; k < kBins; k += BLK) S.hist[k] = 0u;
        __syncthreads();
        stream_rounds<BLK, UF>(dref, n_src, -1.f, [&](const float *dd, int) {
#pragma unroll
          for (int u = 0; u < UF; ++u)
            if (member(dd[u])) atomicAdd(&S.hist[fbin(dd[u])], 1u);
        });
        __syncthreads();
        if (tid == 0) {
          // entries in decreasing fine-bin order: cursor[b] = first slot of bin b
          unsigned int c = 0;
          for (int bb = kBins - 1; bb >= 0; --bb) {
            S.cursor[bb] = c;
            c += S.hist[bb];
          }
          sh_n = c;
          if (c > (unsigned)cap) st_mode = 1;
        }
        __syncthreads();
        if (st_mode == 0) {
          // the ids first; the points are gathered afterwards in one pass
          // over the shell, all loads in flight at once
          stream_rounds<BLK, UF>(dref, n_src, -1.f, [&](const float *dd, int s0) {
#pragma unroll
            for (int u = 0; u < UF; ++u) {
              int s = s0 + u * BLK + tid;
              if (member(dd[u])) {
                unsigned int pos = atomicAdd(&S.cursor[fbin(dd[u])], 1u);
                if (pos < (unsigned)cap) S.id[pos] = s;
              }
            }
          });
          __syncthreads();
          // (global shell: the entry index becomes the sample id)
          if (from_gs) {
            for (int e = tid; e < (int)sh_n; e += BLK) {
              const int x = S.id[e];
              S.pt[e] = gpt[x];
              S.id[e] = gid[x];
            }
          } else {
            for (int e = tid; e < (int)sh_n; e += BLK) S.pt[e] = D[S.id[e]];
          }
          __syncthreads();
          // upper bound of d_ref over each chunk of 64 entries: the upper edge
          // of the fine bin holding its first entry (the top bin's is rref)
          const int K = (int)sh_n;
          for (int c = tid; c * 64 < K && c < kMaxChunks; c += BLK) {
            const unsigned int e = (unsigned)c * 64u;
            unsigned int acc_n = 0;
            int bb = kBins - 1;
            for (; bb > 0; --bb) {
              if (e < acc_n + S.hist[bb]) break;
              acc_n += S.hist[bb];
            }
            S.chunk_ub[c] = (bb >= kBins - 1 || !fine) ? rref : flo + (float)(bb + 1) * fw;
          }
        }
        __syncthreads();
      }
    }
    if (global || st_mode == 1) {
      // ---------------------------------------------------- global-scan steps
      // every feasible sample, all waves; a bounded number of steps per stage
      float4 C = Cref;
      int i = i0;
      int par = 0;
      if (tid == 0) ++sdg.n_global;
      const int i_end = no_prune ? T : (early ? min(T, kEarlySteps) : min(T, i0 + kGlobalSteps - 1));
      while (i <= i_end) {
        float bk = -1.f;
        int bi = INT32_MAX;
        stream_rounds<BLK>(D, M, make_float4(-2.f, 0.f, 0.f, 0.f), [&](const float4 *a, int s0) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            int s = s0 + u * BLK + tid;
            if (s < M && feasible_pt(a[u], chain)) {
              float k = sqdist(C, a[u], chain);
              if (better(k, s, bk, bi)) {
                bk = k;
                bi = s;
              }
            }
          }
        });
        float wk;
        int wi;
        wave_argmax(bk, bi, wk, wi);
        if (lane == 0) {
          S.red_k[par][wave] = wk;
          S.red_i[par][wave] = wi;
        }
        __syncthreads();
        bk = S.red_k[par][0];
        bi = S.red_i[par][0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
          if (better(S.red_k[par][w], S.red_i[par][w], bk, bi)) {
            bk = S.red_k[par][w];
            bi = S.red_i[par][w];
          }
        par ^= 1;
        if (CHAIN == 0 && tid == 0 && (i - 1) % ck == 0) ckq[(i - 1) / ck] = C;
        C = geodesic_step(C, D[bi], i, chain);
        if (tid == 0) tr[2 * (i - 1)] = bi;
        if (i > T - avg && wave == 0) accumulate_iterate(C, chain, acc);
        ++i;
      }
      if (tid == 0) {
        st_C = C;
        st_i = i;
      }
      __syncthreads();
      stalled = false;
    } else {
      // ---------------------------------------------------------- shell steps
      // Entries sit in chunks of 64 (one entry per lane) in decreasing fine
      // bins of d_ref.  Each lane keeps its own best (key, id, point), one
      // wavefront reduction per step of the scan, and the scan stops once no
      // later chunk can beat the best found.  The first two chunks, which
      // almost every step needs, stay in registers for the whole stage (lanes
      // past the shell's end hold copies of entry 0, which change no argmax);
      // later chunks are read from LDS.  When a step needs many chunks the
      // centre has drifted from C_ref: the stage ends and the next one
      // rescans there.
      //
      // Steps run in segments of two kinds.  Sequential segments run in wave
      // 0 alone.  A single wavefront issues about one instruction every few
      // cycles whatever the dependences, so the common step (the first chunk,
      // or the first two once one has often not sufficed in this stage,
      // bounds all others and one lane holds the maximum) is one straight
      // path: 1/i comes from a per-lane table of the next 64 values, and the
      // winners' ids are collected one per lane and written 64 at a time.
      //
      // Late in the descent the winners cycle among a few samples (the
      // support of the ball).  Wave 0 keeps the last distinct winners (up to
      // 8, one per lane); once no new one has appeared for a while, a
      // pipelined segment takes over: wave 0 runs the descent ahead, taking
      // as the winner of each step the one of those candidates farthest from
      // its iterate (a cheap key that only has to predict), kPipeSteps steps
      // per round, and leaves each step's starting iterate and predicted
      // winner in LDS, while the other waves check the steps of the previous
      // round with the full argmax of a sequential step.  Rounds end at a
      // workgroup barrier.  Every iterate wave 0 computes from verified
      // predictions is the one the sequential descent computes (same inputs,
      // same arithmetic), so the trace and the centre are unchanged; at the
      // first step whose prediction fails, the segment ends with that step's
      // starting iterate and a sequential segment redoes the step.
      const int K = (int)sh_n;
      const float theta = st_theta;
      const float slack = 4e-6f * st_rref + 1e-30f;
      const int nchunks = (K + 63) / 64;
      const float4 p0 = S.pt[lane < K ? lane : 0], p1 = S.pt[64 + lane < K ? 64 + lane : 0];
      const int q0 = S.id[lane < K ? lane : 0], q1 = S.id[64 + lane < K ? 64 + lane : 0];
      const float ub1 = nchunks > 1 ? S.chunk_ub[1] : 0.f;
      const float ub2 = nchunks > 2 ? S.chunk_ub[2] : 0.f;
      // the one bound a common step checks: entries past the chunks it
      // scanned, else samples outside the shell, else none
      const bool need_ub1 = nchunks > 1 || theta >= 0.f, need_ub2 = nchunks > 2 || theta >= 0.f;
      const float ubf1 = nchunks > 1 ? ub1 : theta, ubf2 = nchunks > 2 ? ub2 : theta;
      // distance of C from C_ref, compared squared in the bounds (the raw
      // square root is within the slack).  Rotation: |C + C_ref|^2 = 4 -
      // |C - C_ref|^2 for unit quaternions (C stays near C_ref within a stage;
      // the form only feeds bounds).
      auto drift = [&](float4 Cc) {
        float dC2;
        if (CHAIN == 0) {
          const float e0 = Cc.x - Cref.x, e1 = Cc.y - Cref.y, e2 = Cc.z - Cref.z, e3 = Cc.w - Cref.w;
          const float xc = fmaf(e3, e3, fmaf(e2, e2, fmaf(e1, e1, e0 * e0)));
          dC2 = (2.f * xc) * (4.f - xc);
        } else {
          dC2 = sqdist(Cc, Cref, chain);
        }
        return __builtin_amdgcn_sqrtf(dC2);
      };
      // wave-0 state carried across the segments of the stage
      float4 C = Cref;
      int i = i0;
      int misses = 0;                // one-chunk steps that needed more
      bool wide = false, ended = false;
      int backoff = kPipeMinSeq;     // steps with no new winner before a pipelined segment
      const int last_plain = T - avg;  // steps after this one accumulate their iterate
      // wave 0: candidate winners in lanes 0..7 (id -1: empty, its point C_ref,
      // which is never the farthest), the slot the next new winner takes, and
      // the steps since a new winner appeared
      int cand_id = -1;
      float4 cand_p = Cref;
      int nins = 0, stable = 0;
      int last_w = -1;  // winner of the last sequential step
      while (true) {
        if (wave == 0) {
          int ib = i;                                 // first step of the block of 64
          float inv_tab = 1.f / (float)(ib + lane);   // 1/i of step ib + lane
          int trv = 0;                                // winner of step ib + lane
          bool piped = false;
          int next_ck = (i - 1 + ck - 1) / ck * ck;   // next iterate index kept as a checkpoint
          int q_next = next_ck / ck;
          // Steps of the segment up to step `end` with WIDTH chunks in the
          // common step and (SHORT) the short sin/cos series of the geodesic
          // step; returns kStageEnds, kGoWide when one-chunk steps often
          // needed more and the stage should go on with two, kPipe when no
          // new winner has appeared for `backoff` steps and enough steps
          // remain for a pipelined segment, or kRangeDone at `end`.
          constexpr int kStageEnds = 0, kGoWide = 1, kRangeDone = 2, kPipe = 3;
          auto run_steps = [&](auto width, auto short_series, auto accumulate, int end) -> int {
            constexpr int W = decltype(width)::value;
            constexpr bool SHORT = decltype(short_series)::value;
            constexpr bool ACC = decltype(accumulate)::value;  // within the last avg steps
            while (i <= end) {
              if (i - ib == 64) {
                tr[2 * (ib - 1 + lane)] = trv;
                ib = i;
                inv_tab = 1.f / (float)(ib + lane);
              }
              const float inv = readlane_f(inv_tab, i - ib);
              const float dC = drift(C);
              auto beats = [&](float key, float ub) {
                const float b = ub + dC + slack;
                return key > b * b;
              };
              float bk = sqdist(C, p0, chain), bp_x = p0.x, bp_y = p0.y, bp_z = p0.z, bp_w = p0.w;
              int bi = q0;
              auto take = [&](float k, int q, float4 pp) {
                const bool t = (k > bk) | ((k == bk) & (q < bi));
                bk = t ? k : bk;
                bi = t ? q : bi;
                bp_x = t ? pp.x : bp_x;
                bp_y = t ? pp.y : bp_y;
                bp_z = t ? pp.z : bp_z;
                bp_w = t ? pp.w : bp_w;
              };
              int g = W;  // chunks scanned
              if (W == 2) take(sqdist(C, p1, chain), q1, p1);
              float wk = wave_max_key(bk);
              unsigned long long win = __ballot(bk == wk);
              const bool bounded = W == 2 ? (!need_ub2 || beats(wk, ubf2)) : (!need_ub1 || beats(wk, ubf1));
              if (!(bounded && __popcll(win) == 1)) {
                // -------------------------------------------- uncommon step
                if (W == 1 && nchunks > 1 && !beats(wk, ub1)) {
                  take(sqdist(C, p1, chain), q1, p1);
                  wk = wave_max_key(bk);
                  g = 2;
                }
                if (g == 2 && nchunks > 2 && !beats(wk, ub2)) {
                  float4 p = S.pt[2 * 64 + lane];
                  int q = S.id[2 * 64 + lane];
                  while (true) {
                    float4 np;
                    int nq;
                    const bool more = g + 1 < nchunks;
                    if (more) {
                      np = S.pt[(g + 1) * 64 + lane];
                      nq = S.id[(g + 1) * 64 + lane];
                    }
                    const float kk = sqdist(C, p, chain);
                    take(g * 64 + lane < K ? kk : -1.f, q, p);
                    wk = wave_max_key(bk);
                    ++g;
                    if (!more || beats(wk, S.chunk_ub[g])) break;
                    p = np;
                    q = nq;
                  }
                }
                if (theta >= 0.f && !beats(wk, theta)) {
                  stage_groups += g;
                  return kStageEnds;  // the shell no longer suffices
                }
                // winner: the one lane holding the maximum key, else (a tie)
                // the lowest sample id among the lanes that hold it
                win = __ballot(bk == wk);
                if (__popcll(win) > 1) {
                  const int wmin = wave_min_i32(bk == wk ? bi : INT32_MAX);
                  win = __ballot(bk == wk && bi == wmin);
                }
              }
              stage_groups += g;
              const int wl = (int)__ffsll((long long)win) - 1;
              const int wi = __builtin_amdgcn_readlane(bi, wl);
              const float4 pt = make_float4(readlane_f(bp_x, wl), readlane_f(bp_y, wl), readlane_f(bp_z, wl),
                                            readlane_f(bp_w, wl));
              if (CHAIN == 0 && i - 1 == next_ck) {
                if (lane == 0) ckq[q_next] = C;
                next_ck += ck;
                ++q_next;
              }
              C = geodesic_step_inv<SHORT>(C, pt, inv, chain);
              trv = lane == i - ib ? wi : trv;
              if (ACC) accumulate_iterate(C, chain, acc);
              ++i;
              if (SHORT && !ACC) {
                last_w = wi;
                const bool known = (__ballot(cand_id == wi) & 0xFFull) != 0ull;
                const bool ins = !known && lane == nins;
                cand_id = ins ? wi : cand_id;
                cand_p = make_float4(ins ? pt.x : cand_p.x, ins ? pt.y : cand_p.y, ins ? pt.z : cand_p.z,
                                     ins ? pt.w : cand_p.w);
                nins = known ? nins : ((nins + 1) & 7);
                stable = known ? stable + 1 : 0;
              }
              if (g > recentre && i - i0 > kMinShellSteps) return kStageEnds;  // re-centre the shell
              if (W == 1 && g > 1 && ++misses * 4 > i - i0 && i - i0 >= 16) return kGoWide;
              if (SHORT && !ACC && stable >= backoff && end - i + 1 >= 2 * kPipeSteps) return kPipe;
            }
            return kRangeDone;
          };
          // Ranges of steps with no per-step choice of the sin/cos series or
          // of accumulating the iterate: before kShortSeriesStep, then the
          // rest, each split at the last avg steps.
          auto run_range = [&](auto short_series, auto accumulate, int end) {
            if (ended || piped || i > end) return;
            int r = wide ? run_steps(std::integral_constant<int, 2>(), short_series, accumulate, end)
                         : run_steps(std::integral_constant<int, 1>(), short_series, accumulate, end);
            if (r == kGoWide) {
              wide = true;
              r = run_steps(std::integral_constant<int, 2>(), short_series, accumulate, end);
            }
            ended = r == kStageEnds;
            piped = r == kPipe;
          };
          const int long_end = min(T, kShortSeriesStep - 1);
          run_range(std::false_type(), std::false_type(), min(long_end, last_plain));
          run_range(std::false_type(), std::true_type(), long_end);
          run_range(std::true_type(), std::false_type(), last_plain);
          run_range(std::true_type(), std::true_type(), T);
          if (lane < i - ib) tr[2 * (ib - 1 + lane)] = trv;
          if (lane == 0) sdg.n_groups += stage_groups;
          stage_groups = 0;
          if (lane == 0) {
            st_C = C;
            st_i = i;
            pl_go = piped ? 1 : 0;
          }
          for (int k = lane; k < 3; k += 64) pl_fail[k] = INT32_MAX;
        }
        __syncthreads();
        if (!pl_go) break;
        // ------------------------------------------------ pipelined segment
        const int pi0 = st_i, pend = last_plain;
        const int nrounds = (pend - pi0 + kPipeSteps) / kPipeSteps;
        float4 Cs = st_C;                       // wave 0: the iterate ahead
        float4 cv = Cs;                         // wave 0: starting iterate of step (round start + lane)
        int pv = 0;                             // wave 0: predicted winner of that step
        int fail_step = INT32_MAX;
        float4 fail_C = Cs;
        // wave 0: when only two samples have won since the stage began the
        // winners alternate; the first predicted winner is then the one not
        // taken last
        const unsigned long long vm = __ballot(cand_id >= 0) & 0xFFull;
        const bool two = __popcll(vm) == 2;
        const int l0 = (int)__ffsll((long long)vm) - 1, l1 = (int)__ffsll((long long)(vm & (vm - 1ull))) - 1;
        const bool zero_last = __builtin_amdgcn_readlane(cand_id, two ? l0 : 0) == last_w;
        const int la = two ? (zero_last ? l1 : l0) : 0, lb = two ? (zero_last ? l0 : l1) : 0;
        const int idA = __builtin_amdgcn_readlane(cand_id, la), idB = __builtin_amdgcn_readlane(cand_id, lb);
        const float4 pA = make_float4(readlane_f(cand_p.x, la), readlane_f(cand_p.y, la), readlane_f(cand_p.z, la),
                                      readlane_f(cand_p.w, la));
        const float4 pB = make_float4(readlane_f(cand_p.x, lb), readlane_f(cand_p.y, lb), readlane_f(cand_p.z, lb),
                                      readlane_f(cand_p.w, lb));
        for (int r = 0; r <= nrounds; ++r) {
          const int s_r = pi0 + r * kPipeSteps;
          const int slot = r % 3;
          if (tid == 0) pl_fail[slot] = INT32_MAX;  // (read last at the start of round r - 2)
          if (wave == 0) {
            if (r < nrounds) {
              const int n_r = min(kPipeSteps, pend - s_r + 1);
              const float pinv_tab = 1.f / (float)(s_r + lane);  // 1/i of step s_r + lane
              // (kPipeSteps is even: step k of every round takes A when k is even)
              if (two) {
                for (int k = 0; k < n_r; ++k) {
                  const float inv = readlane_f(pinv_tab, k);
                  const bool odd = (k & 1) != 0;
                  const float4 pp = odd ? pB : pA;
                  const bool mine = lane == k;
                  cv = make_float4(mine ? Cs.x : cv.x, mine ? Cs.y : cv.y, mine ? Cs.z : cv.z, mine ? Cs.w : cv.w);
                  pv = mine ? (odd ? idB : idA) : pv;
                  Cs = geodesic_step_inv<true>(Cs, pp, inv, chain);
                }
              } else
              for (int k = 0; k < n_r; ++k) {
                const float inv = readlane_f(pinv_tab, k);
                // predicted winner: the argmax over the candidates (lanes
                // 0..7) with the keys and tie rule of the full argmax, near
                // convergence the candidates being almost equidistant
                // The step toward every candidate, one per lane, alongside
                // the argmax (sharing the chords of the keys): the winner's
                // lane holds bitwise the step toward the winner.  For the
                // rotation chain the stages of the step are placed between
                // those of the argmax's reduction (scheduling barriers), so
                // that the two dependent chains overlap in the one wave.
                float u;
                float4 Cn;
                int ub;
                if constexpr (CHAIN == 0) {
                  float x, y;
                  rot_chord_sq(Cs, cand_p, x, y);
                  u = (2.f * x) * y;  // the key of sqdist
                  ub = __float_as_int(u);
                  ub = max(ub, __builtin_amdgcn_update_dpp(INT32_MIN, ub, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
                  // (the empty asm statements keep each stage where it is
                  // written: without them the compiler moves the step's
                  // stages below the argmax, to their first use)
                  RotChords rc = rot_chords(x, y);
                  __asm__ volatile("" : "+v"(rc.xs), "+v"(rc.rx), "+v"(rc.ry));
                  __builtin_amdgcn_sched_barrier(0);
                  ub = max(ub, __builtin_amdgcn_update_dpp(INT32_MIN, ub, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
                  float th = rot_step_angle(rc, inv);
                  __asm__ volatile("" : "+v"(th));
                  __builtin_amdgcn_sched_barrier(0);
                  ub = max(ub, __builtin_amdgcn_update_dpp(INT32_MIN, ub, 0x141, 0xF, 0xF, false));  // row_half_mirror
                  Cn = rot_interp<true>(rc, th, Cs, cand_p);
                  __asm__ volatile("" : "+v"(Cn.x), "+v"(Cn.y), "+v"(Cn.z), "+v"(Cn.w));
                } else {
                  u = sqdist(Cs, cand_p, chain);
                  Cn = geodesic_step_inv<true>(Cs, cand_p, inv, chain);
                  ub = __float_as_int(u);
                  ub = max(ub, __builtin_amdgcn_update_dpp(INT32_MIN, ub, 0xB1, 0xF, 0xF, false));
                  ub = max(ub, __builtin_amdgcn_update_dpp(INT32_MIN, ub, 0x4E, 0xF, 0xF, false));
                  ub = max(ub, __builtin_amdgcn_update_dpp(INT32_MIN, ub, 0x141, 0xF, 0xF, false));
                }
                const int umax = __builtin_amdgcn_readlane(ub, 0);
                const bool at_max = __float_as_int(u) == umax;
                unsigned long long tie = __ballot(at_max) & 0xFFull;
                if (__popcll(tie) > 1) {  // equal keys: the lowest sample id
                  int iv = at_max ? cand_id : INT32_MAX;
                  iv = min(iv, __builtin_amdgcn_update_dpp(INT32_MAX, iv, 0xB1, 0xF, 0xF, false));
                  iv = min(iv, __builtin_amdgcn_update_dpp(INT32_MAX, iv, 0x4E, 0xF, 0xF, false));
                  iv = min(iv, __builtin_amdgcn_update_dpp(INT32_MAX, iv, 0x141, 0xF, 0xF, false));
                  const int imin = __builtin_amdgcn_readlane(iv, 0);
                  tie = __ballot(at_max && cand_id == imin) & 0xFFull;
                }
                const int wl = (int)__ffsll((long long)tie) - 1;
                const int pid = __builtin_amdgcn_readlane(cand_id, wl);
                const bool mine = lane == k;
                cv = make_float4(mine ? Cs.x : cv.x, mine ? Cs.y : cv.y, mine ? Cs.z : cv.z, mine ? Cs.w : cv.w);
                pv = mine ? pid : pv;
                Cs = make_float4(readlane_f(Cn.x, wl), readlane_f(Cn.y, wl), readlane_f(Cn.z, wl), readlane_f(Cn.w, wl));
              }
              if (lane < n_r) {
                pl_C[slot][lane] = cv;
                pl_W[slot][lane] = pv;
                // (a checkpoint from a step found wrong later is rewritten
                // when the step is redone)
                const int im1 = s_r + lane - 1;
                if (CHAIN == 0 && im1 % ck == 0) ckq[im1 / ck] = cv;
              }
              if (r == nrounds - 1 && lane == 0) pl_Cend = Cs;
            }
          } else if (r >= 1 && wave != kSkipWave) {
            // check the steps of round r - 1, one wave per step
            const int s_p = s_r - kPipeSteps, n_p = min(kPipeSteps, pend - s_p + 1);
            const int pslot = (r + 2) % 3;
            const int vw = wave < kSkipWave ? wave - 1 : wave - 2;
            for (int k = vw; k < n_p; k += kVerifiers) {
              const float4 Cv = pl_C[pslot][k];
              const int pid = pl_W[pslot][k];
              const float dC = drift(Cv);
              auto beats = [&](float key, float ub) {
                const float b = ub + dC + slack;
                return key > b * b;
              };
              float bk = sqdist(Cv, p0, chain);
              int bi = q0;
              auto take = [&](float kk, int q) {
                const bool t = (kk > bk) | ((kk == bk) & (q < bi));
                bk = t ? kk : bk;
                bi = t ? q : bi;
              };
              take(sqdist(Cv, p1, chain), q1);
              float wk = wave_max_key(bk);
              bool ok = true;
              if (need_ub2 && !beats(wk, ubf2)) {
                // further chunks until one bounds the rest, then the samples
                // outside the shell
                int g = 2;
                while (g < nchunks) {
                  const float4 p = S.pt[g * 64 + lane];
                  const int q = S.id[g * 64 + lane];
                  take(g * 64 + lane < K ? sqdist(Cv, p, chain) : -1.f, q);
                  wk = wave_max_key(bk);
                  ++g;
                  if (g < nchunks && beats(wk, S.chunk_ub[g])) break;
                }
                if (theta >= 0.f && !beats(wk, theta)) ok = false;
                // a step that needs many chunks goes to a sequential segment,
                // which re-centres the shell
                if (g > recentre && s_p + k - i0 > kMinShellSteps) ok = false;
              }
              if (ok) {
                const unsigned long long win = __ballot(bk == wk);
                const int wi = __popcll(win) > 1 ? wave_min_i32(bk == wk ? bi : INT32_MAX)
                                                 : __builtin_amdgcn_readlane(bi, (int)__ffsll((long long)win) - 1);
                ok = wi == pid;
              }
              if (!ok && lane == 0) atomicMin(&pl_fail[pslot], k);
            }
          }
          __syncthreads();
          if (r >= 1) {
            const int s_p = s_r - kPipeSteps, n_p = min(kPipeSteps, pend - s_p + 1);
            const int pslot = (r + 2) % 3;
            const int f = pl_fail[pslot];
            // the verified steps of round r - 1 enter the trace
            if (wave == 1 && lane < min(n_p, f)) tr[2 * (s_p + lane - 1)] = pl_W[pslot][lane];
            if (f != INT32_MAX) {
              fail_step = s_p + f;
              fail_C = pl_C[pslot][f];
              break;
            }
          }
        }
        if (tid == 0) {
          ++sdg.n_seg;
          sdg.n_piped += (fail_step == INT32_MAX ? pend + 1 : fail_step) - pi0;
          sdg.n_fail += fail_step == INT32_MAX ? 0 : 1;
        }
        if (fail_step == INT32_MAX) {
          C = pl_Cend;
          i = pend + 1;
        } else {
          C = fail_C;
          i = fail_step;
          backoff = min(2 * backoff, kPipeMaxSeq);
          stable = 0;
        }
        // (pl_Cend and the failing slot are read before any later write:
        // the next write to either follows the barrier that ends the next
        // sequential segment)
      }
      // a stage that made no step: with the global shell, rescan every
      // sample next; else a stage of full scans
      stalled = st_i == i0 && !use_gs;
      if (st_i == i0) use_gs = false;
    }
  }
  // ------------------------------------------------------------------ centre
  if (tid == 0) {
    rec[j].n_rescan[chain] = sdg.n_rescan;
    rec[j].n_global[chain] = sdg.n_global | (sg.n_built << 16);
    rec[j].n_groups[chain] = sdg.n_groups;
    // (the real-time clock runs at 100 MHz)
    rec[j].chain_us[chain] = (int32_t)((__builtin_amdgcn_s_memrealtime() - sdg.t_start) / 100ull);
    if (chain == 0) {
      rec[j].n_piped = sdg.n_piped;
      rec[j].n_pipe_fail = sdg.n_fail;
      rec[j].n_pipe_seg = sdg.n_seg;
    }
    if (chain == 0) {
      double Md[9], Rd[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Md[k] = (double)acc[k];
      polar_so3<double>(Md, Rd, 12);
#pragma unroll
      for (int k = 0; k < 9; ++k) rec[j].centre[k] = (float)Rd[k];
    } else {
      const int na = avg < T ? avg : T;
#pragma unroll
      for (int k = 0; k < 3; ++k) rec[j].centre[9 + k] = acc[k] / (float)na;
    }
  }
}

// One workgroup of chain_block<V>() threads per (instance, chain): even blocks
// run the rotation chain, odd blocks the translation chain.
// The narrow variant is held to 128 VGPRs (a few spills outside the step
// loops), so that four chains share a compute unit: a chain's steps run in
// one wavefront, which leaves most issue slots to the other chains' waves.
template <int V>
__global__ void __launch_bounds__(chain_block<V>(), V == kChainWide ? 1 : 4) k_megb_chain(const int64_t *__restrict__ sample_off, int64_t max_m,
                                                            const float4 *__restrict__ quat,
                                                            const float4 *__restrict__ trans, MegbRec *rec,
                                                            float *dref_all, int64_t total_samples,
                                                            int32_t *trace, float4 *ckpt, int ck, int T, int avg,
                                                            int cap, int no_prune, int32_t *gid,
                                                            float4 *gpt, int64_t gstride) {
  extern __shared__ float4 sh_pt[];
  __shared__ unsigned int hist[kBins];
  __shared__ unsigned int cursor[kBins];
  __shared__ float chunk_ub[kMaxChunks];
  __shared__ float red_k[2][kChainWaves];
  __shared__ int red_i[2][kChainWaves];
  const ChainShared S{sh_pt, reinterpret_cast<int *>(sh_pt + cap), hist, cursor, chunk_ub, red_k, red_i};
  if (blockIdx.x & 1)
    chain_run<1, V>(S, sample_off, max_m, trans, rec, dref_all, total_samples, trace, ckpt, ck, T, avg, cap,
                       no_prune, gid, gpt, gstride);
  else
    chain_run<0, V>(S, sample_off, max_m, quat, rec, dref_all, total_samples, trace, ckpt, ck, T, avg, cap,
                       no_prune, gid, gpt, gstride);
}

// float64 radii about the centre: max ||R* - R_s||_F^2 and ||t* - t_s||^2.
template <int PER>
__global__ void __launch_bounds__(kBlock) k_megb_radii(const int64_t *__restrict__ sample_off, int64_t total,
                                                       int64_t max_m, const float *__restrict__ poses,
                                                       const uint8_t *__restrict__ mask, MegbRec *rec) {
  const int j = blockIdx.y;
  int64_t off, M;
  sample_range(sample_off, j, total, max_m, off, M);
  const int64_t s0 = (int64_t)blockIdx.x * (kBlock * PER) + threadIdx.x;
  __shared__ double red[2][kWaves];
  double fr = 0.0, ft = 0.0;
  if (rec[j].first != INT32_MAX) {
    // PER samples per thread, kBlock apart, loads in flight together
    uint8_t m[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t s = s0 + u * kBlock;
      m[u] = s < M ? mask[off + s] : (uint8_t)0;
    }
    float4 pa[PER], pb[PER], pc[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t s = s0 + u * kBlock;
      if (s < M && (m[u] & PURSE_MASK_FEASIBLE)) {
        const float4 *pp = reinterpret_cast<const float4 *>(poses + 12 * (off + s));
        pa[u] = pp[0];
        pb[u] = pp[1];
        pc[u] = pp[2];
      }
    }
    const float *C = rec[j].centre;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t s = s0 + u * kBlock;
      if (s < M && (m[u] & PURSE_MASK_FEASIBLE)) {
        const float P[12] = {pa[u].x, pa[u].y, pa[u].z, pa[u].w, pb[u].x, pb[u].y,
                             pb[u].z, pb[u].w, pc[u].x, pc[u].y, pc[u].z, pc[u].w};
        double r = 0.0, t = 0.0;
        for (int k = 0; k < 9; ++k) {
          double d = (double)C[k] - (double)P[k];
          r += d * d;
        }
        for (int k = 9; k < 12; ++k) {
          double d = (double)C[k] - (double)P[k];
          t += d * d;
        }
        fr = fmax(fr, r);
        ft = fmax(ft, t);
      }
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    fr = fmax(fr, __shfl_xor(fr, o, 64));
    ft = fmax(ft, __shfl_xor(ft, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = fr;
    red[1][w] = ft;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWaves; ++k) {
      fr = fmax(fr, red[0][k]);
      ft = fmax(ft, red[1][k]);
    }
    fr = fmax(fr, red[0][0]);
    ft = fmax(ft, red[1][0]);
    if (fr > 0.0) atomicMax(&rec[j].max_rot, (unsigned long long)__double_as_longlong(fr));
    if (ft > 0.0) atomicMax(&rec[j].max_trans, (unsigned long long)__double_as_longlong(ft));
  }
}

// Signature of each instance's descent, stored with the checkpoints it left,
// so that the backward uses them only for this descent: the sum of a term
// per step of (step, winner, the bits of the winner's rotation), and one for
// the start (the first feasible sample), which determine the iterates.
__global__ void __launch_bounds__(kBlock) k_megb_sign(const int64_t *__restrict__ sample_off, int64_t total,
                                                      int64_t max_m, const float *__restrict__ poses,
                                                      const int32_t *__restrict__ trace, MegbRec *rec, int T, int ck) {
  const int j = blockIdx.x;
  int64_t off, M;
  sample_range(sample_off, j, total, max_m, off, M);
  const int first = rec[j].first;
  const int32_t *tr = trace + (int64_t)j * T * 2;
  unsigned long long h = 0ull;
  if (first != INT32_MAX)
    for (int i = (int)threadIdx.x; i <= T; i += kBlock) {
      const int id = i == 0 ? first : tr[2 * (i - 1)];
      if (id >= 0 && id < M) {
        uint32_t R[9];
        const float *P = poses + 12 * (off + id);
        for (int k = 0; k < 9; ++k) R[k] = __float_as_uint(P[k]);
        h += step_sig_term(i, id, R);
      } else {
        h += trace_mix(i, id);
      }
    }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
  __shared__ unsigned long long part[kWaves];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0ull;
    for (int w = 0; w < kWaves; ++w) t += part[w];
    rec[j].ck_hash = t;
    rec[j].ck_T = first != INT32_MAX ? T : 0;
    rec[j].ck_every = ck;
  }
}

// ---------------------------------------------------------------------------
// Step III of the paper ("The CLOSURE Algorithm"): the exact minimum enclosing
// ball of the feasible samples, translations in R^3 and rotations as unit
// quaternions in R^4 put on one hemisphere (the quaternions of the descent's
// centre and of every sample with a non-negative inner product), replacing
// the descent's centre.  One workgroup per (instance, chain), float64.
//
// The support of the exact ball lies among the samples farthest from the
// descent's centre, which is close to the exact one: a shell of the
// farthest samples (a 256-bin histogram of their distance picks a threshold
// that keeps at most kExactShell of them) is staged in LDS and its exact
// ball found by support-set iteration: the support set B (at most dim + 1
// points) and its ball; the shell's farthest point p from the centre, if
// outside, gives the new ball as the smallest ball enclosing B and p whose
// boundary holds p and some subset of B (the lanes try the 2^|B| subsets,
// each by the circumsphere of its points in their affine hull).  The radius
// grows at every step and the support sets are finite, so this ends; the
// last ball encloses the shell and is the ball of a subset of it, hence the
// shell's minimum ball.  Every sample is then checked against it; any sample
// outside is added to the shell and the iteration resumes, so the final ball
// encloses all samples and is the minimum ball of a subset: the exact one.
constexpr int kExactShell = 1024;   // staged at first
constexpr int kExactCap = 2048;     // shell capacity including samples added by the checks
constexpr int kExactRounds = 16;    // check-and-add rounds before giving up (the descent's centre is kept)
constexpr int kExactBins = 256;

__device__ __forceinline__ void exact_point(const float4 *D, int64_t s, int chain, const double ref[4], double x[4]) {
  const float4 a = D[s];
  if (chain == 0) {
    x[0] = a.x;
    x[1] = a.y;
    x[2] = a.z;
    x[3] = a.w;
    const double dot = x[0] * ref[0] + x[1] * ref[1] + x[2] * ref[2] + x[3] * ref[3];
    if (dot < 0.0)
      for (int k = 0; k < 4; ++k) x[k] = -x[k];
  } else {
    x[0] = a.x;
    x[1] = a.y;
    x[2] = a.z;
    x[3] = 0.0;
  }
}

__device__ __forceinline__ double exact_d2(const double x[4], const double c[4]) {
  double d = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) d += (x[k] - c[k]) * (x[k] - c[k]);
  return d;
}

// Circumsphere of k points P[0..k) (rows of 4) in their affine hull:
// c = P0 + sum lam_i (P_i - P0) with 2 (P_i - P0).(c - P0) = |P_i - P0|^2.
// Returns false for affinely dependent points.
__device__ __forceinline__ bool exact_circumsphere(const double P[5][4], int k, double c[4], double &r2) {
  double A[4][4], G[4][4], b[4], lam[4];
  const int m = k - 1;
  for (int i = 0; i < m; ++i)
    for (int q = 0; q < 4; ++q) A[i][q] = P[i + 1][q] - P[0][q];
  for (int i = 0; i < m; ++i) {
    b[i] = 0.0;
    for (int q = 0; q < 4; ++q) b[i] += 0.5 * A[i][q] * A[i][q];
    for (int jj = 0; jj < m; ++jj) {
      double g = 0.0;
      for (int q = 0; q < 4; ++q) g += A[i][q] * A[jj][q];
      G[i][jj] = g;
    }
  }
  // Cholesky of the Gram matrix (positive definite iff independent)
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = fmax(scale, G[i][i]);
  for (int i = 0; i < m; ++i) {
    for (int jj = 0; jj <= i; ++jj) {
      double v = G[i][jj];
      for (int q = 0; q < jj; ++q) v -= G[i][q] * G[jj][q];
      if (i == jj) {
        if (!(v > 1e-14 * scale)) return false;
        G[i][i] = sqrt(v);
      } else {
        G[i][jj] = v / G[jj][jj];
      }
    }
  }
  for (int i = 0; i < m; ++i) {
    double v = b[i];
    for (int q = 0; q < i; ++q) v -= G[i][q] * lam[q];
    lam[i] = v / G[i][i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double v = lam[i];
    for (int q = i + 1; q < m; ++q) v -= G[q][i] * lam[q];
    lam[i] = v / G[i][i];
  }
  for (int q = 0; q < 4; ++q) {
    double v = P[0][q];
    for (int i = 0; i < m; ++i) v += lam[i] * A[i][q];
    c[q] = v;
  }
  r2 = exact_d2(P[0], c);
  return true;
}

__global__ void __launch_bounds__(kBlock) k_megb_exact(const int64_t *__restrict__ sample_off, int64_t total,
                                                       int64_t max_m, const float4 *__restrict__ quat,
                                                       const float4 *__restrict__ trans, MegbRec *rec) {
  const int j = blockIdx.x >> 1, chain = blockIdx.x & 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t off, M64;
  sample_range(sample_off, j, total, max_m, off, M64);
  const int M = (int)M64;
  if (rec[j].first == INT32_MAX) return;  // empty instance (whole workgroup)
  const float4 *D = (chain ? trans : quat) + off;
  const int dim = chain ? 3 : 4;
  __shared__ double pts[kExactCap][4];
  __shared__ int hist[kExactBins];
  __shared__ int n_s, fail_s, nb_s, add_s;
  __shared__ double B_s[5][4], c_s[4], r2_s, thr_s;
  __shared__ double red_v[kWaves];
  __shared__ int red_i[kWaves];
  // the descent's centre (and the hemisphere's reference)
  double ref[4];
  {
    const float *C = rec[j].centre;
    if (chain == 0) {
      const float4 q = quat_from_rot(C);
      ref[0] = q.x;
      ref[1] = q.y;
      ref[2] = q.z;
      ref[3] = q.w;
    } else {
      ref[0] = C[9];
      ref[1] = C[10];
      ref[2] = C[11];
      ref[3] = 0.0;
    }
  }
  // ---- largest distance from the descent's centre, then the shell threshold
  auto block_max = [&](double v, int i, double &bv, int &bi) {
    for (int o = 32; o >= 1; o >>= 1) {
      const double v2 = __shfl_xor(v, o, 64);
      const int i2 = __shfl_xor(i, o, 64);
      if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
      }
    }
    if (lane == 0) {
      red_v[wave] = v;
      red_i[wave] = i;
    }
    __syncthreads();
    bv = red_v[0];
    bi = red_i[0];
    for (int w = 1; w < kWaves; ++w)
      if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < bi)) {
        bv = red_v[w];
        bi = red_i[w];
      }
    __syncthreads();
  };
  double dmax = -1.0;
  int imax = INT32_MAX;
  for (int s = tid; s < M; s += kBlock) {
    if (!feasible_pt(D[s], chain)) continue;
    double x[4];
    exact_point(D, s, chain, ref, x);
    const double d = exact_d2(x, ref);
    if (d > dmax) {
      dmax = d;
      imax = s;
    }
  }
  double r2hat;
  int ihat;
  block_max(dmax, imax, r2hat, ihat);
  const double rhat = sqrt(fmax(r2hat, 0.0));
  for (int k = tid; k < kExactBins; k += kBlock) hist[k] = 0;
  __syncthreads();
  // bins of the distance over [0, rhat]; the threshold keeps at most
  // kExactShell samples (all of them when there are fewer)
  const double binw = rhat > 0.0 ? rhat / kExactBins : 1.0;
  for (int s = tid; s < M; s += kBlock) {
    if (!feasible_pt(D[s], chain)) continue;
    double x[4];
    exact_point(D, s, chain, ref, x);
    const int bin = min(kExactBins - 1, (int)(sqrt(exact_d2(x, ref)) / binw));
    atomicAdd(&hist[bin], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0, b = kExactBins;
    while (b > 0 && acc + hist[b - 1] <= kExactShell) acc += hist[--b];
    thr_s = b == kExactBins ? rhat : b * binw;  // (a top bin over capacity: its farthest sample only)
    n_s = 0;
    fail_s = 0;
  }
  __syncthreads();
  const double thr = thr_s;
  for (int s = tid; s < M; s += kBlock) {
    if (!feasible_pt(D[s], chain)) continue;
    double x[4];
    exact_point(D, s, chain, ref, x);
    if (sqrt(exact_d2(x, ref)) >= thr || s == ihat) {
      const int k = atomicAdd(&n_s, 1);
      if (k < kExactShell)
        for (int q = 0; q < 4; ++q) pts[k][q] = x[q];
    }
  }
  __syncthreads();
  if (tid == 0) {
    n_s = min(n_s, kExactShell);
    // start: the ball of the single farthest sample
    double x[4];
    exact_point(D, ihat, chain, ref, x);
    for (int q = 0; q < 4; ++q) {
      B_s[0][q] = x[q];
      c_s[q] = x[q];
    }
    nb_s = 1;
    r2_s = 0.0;
  }
  __syncthreads();
  const double eps = 1e-12;
  for (int round = 0; round < kExactRounds; ++round) {
    // ---- support-set iteration on the shell
    for (int step = 0; step < 4 * kExactCap; ++step) {
      const double c[4] = {c_s[0], c_s[1], c_s[2], c_s[3]};
      const double r2 = r2_s;
      double bv = -1.0;
      int bi = INT32_MAX;
      for (int k = tid; k < n_s; k += kBlock) {
        const double d = exact_d2(pts[k], c);
        if (d > bv) {
          bv = d;
          bi = k;
        }
      }
      double fv;
      int fi;
      block_max(bv, bi, fv, fi);
      if (fi == INT32_MAX || fv <= r2 * (1.0 + eps) + 1e-300) break;
      // smallest ball with p on its boundary enclosing B and p (wave 0: one
      // subset of B per lane)
      if (wave == 0) {
        const int nb = nb_s;
        double best_r2 = INFINITY, best_c[4] = {0, 0, 0, 0};
        int best_m = -1;
        if (lane < (1 << nb)) {
          double P[5][4];
          int k = 0;
          for (int q = 0; q < 4; ++q) P[k][q] = pts[fi][q];
          ++k;
          for (int i = 0; i < nb; ++i)
            if ((lane >> i) & 1) {
              if (k < dim + 1)
                for (int q = 0; q < 4; ++q) P[k][q] = B_s[i][q];
              ++k;
            }
          double cc[4], rr2;
          if (k <= dim + 1 && exact_circumsphere(P, k, cc, rr2)) {
            bool encl = true;
            for (int i = 0; i < nb; ++i) encl = encl && exact_d2(B_s[i], cc) <= rr2 * (1.0 + 1e-10) + 1e-300;
            if (encl) {
              best_r2 = rr2;
              best_m = lane;
              for (int q = 0; q < 4; ++q) best_c[q] = cc[q];
            }
          }
        }
        // smallest radius, then the lower subset index
        double v = -best_r2;
        int m = best_m < 0 ? INT32_MAX : best_m;
        for (int o = 32; o >= 1; o >>= 1) {
          const double v2 = __shfl_xor(v, o, 64);
          const int m2 = __shfl_xor(m, o, 64);
          if (v2 > v || (v2 == v && m2 < m)) {
            v = v2;
            m = m2;
          }
        }
        if (m == INT32_MAX) {
          if (lane == 0) fail_s = 1;
        } else if (lane == m) {
          double nB[5][4];
          int k = 0;
          for (int q = 0; q < 4; ++q) nB[k][q] = pts[fi][q];
          ++k;
          for (int i = 0; i < nb; ++i)
            if ((m >> i) & 1) {
              for (int q = 0; q < 4; ++q) nB[k][q] = B_s[i][q];
              ++k;
            }
          for (int i = 0; i < k; ++i)
            for (int q = 0; q < 4; ++q) B_s[i][q] = nB[i][q];
          nb_s = k;
          for (int q = 0; q < 4; ++q) c_s[q] = best_c[q];
          r2_s = best_r2;
        }
      }
      __syncthreads();
      if (fail_s) break;
    }
    if (fail_s) break;
    // ---- every sample against the ball; samples outside join the shell
    if (tid == 0) add_s = 0;
    __syncthreads();
    {
      const double c[4] = {c_s[0], c_s[1], c_s[2], c_s[3]};
      const double lim = r2_s * (1.0 + 1e-9) + 1e-300;
      for (int s = tid; s < M; s += kBlock) {
        if (!feasible_pt(D[s], chain)) continue;
        double x[4];
        exact_point(D, s, chain, ref, x);
        if (exact_d2(x, c) > lim) {
          const int k = atomicAdd(&add_s, 1);
          const int slot = n_s + k;
          if (slot < kExactCap)
            for (int q = 0; q < 4; ++q) pts[slot][q] = x[q];
        }
      }
    }
    __syncthreads();
    if (add_s == 0) break;
    if (tid == 0) {
      if (n_s + add_s > kExactCap) fail_s = 1;  // (the shell is full: the descent's centre is kept)
      n_s = min(kExactCap, n_s + add_s);
    }
    __syncthreads();
    if (fail_s) break;
    if (round == kExactRounds - 1 && tid == 0) fail_s = 1;
  }
  __syncthreads();
  if (tid == 0 && !fail_s) {
    if (chain == 0) {
      double q[4] = {c_s[0], c_s[1], c_s[2], c_s[3]};
      const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      if (n > 0.0) {
        const float4 qf = make_float4((float)(q[0] / n), (float)(q[1] / n), (float)(q[2] / n), (float)(q[3] / n));
        float Rr[9];
        rot_from_quat(qf, Rr);
        for (int k = 0; k < 9; ++k) rec[j].centre[k] = Rr[k];
      }
    } else {
      for (int k = 0; k < 3; ++k) rec[j].centre[9 + k] = (float)c_s[k];
    }
  }
}

__global__ void k_megb_final(int n_inst, const MegbRec *rec, float *centre, double *radii, int64_t *n_feasible,
                             int32_t *inst_status) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_inst) return;
  const MegbRec r = rec[j];
  n_feasible[j] = (int64_t)r.n_feasible;
  if (r.first == INT32_MAX) {
    const float nanf_ = __int_as_float(0x7fc00000);
    for (int k = 0; k < 12; ++k) centre[12 * j + k] = nanf_;
    radii[2 * j] = radii[2 * j + 1] = __longlong_as_double(0x7ff8000000000000ll);
    if ((inst_status[j] & 0xFF) == PURSE_INST_OK) inst_status[j] = (inst_status[j] & ~0xFF) | PURSE_INST_EMPTY;
    return;
  }
  for (int k = 0; k < 12; ++k) centre[12 * j + k] = r.centre[k];
  double fr = __longlong_as_double((long long)r.max_rot);
  double ft = __longlong_as_double((long long)r.max_trans);
  double x = sqrt(fr) / (2.0 * sqrt(2.0));
  radii[2 * j] = 2.0 * asin(x < 1.0 ? x : 1.0);
  radii[2 * j + 1] = sqrt(ft);
}

void launch_megb(const DevBatch &b, const DevParams &p, const float *poses, const uint8_t *mask, MegbRec *rec,
                 float4 *quat, float4 *trans, float *dref, float4 *ckpt, EarlyScratch *es, int32_t *gid, float4 *gpt,
                 float *centre, double *radii, int64_t *n_feasible, int32_t *trace, int32_t *inst_status,
                 int64_t max_samples, int64_t total_samples, hipStream_t stream) {
  const int ck = ckpt_spacing(p.ckpt_every);
  const int n = b.n_inst;
  hipLaunchKernelGGL(k_megb_init, dim3((n + 255) / 256), dim3(256), 0, stream, n, rec);
  // (several samples per thread on large instances: fewer workgroups and
  // atomics; one on small ones, whose passes are latency-bound)
  const bool per4 = max_samples >= kPassPerMin;
  const int per = per4 ? kPassPer : 1;
  dim3 grid((unsigned)((max_samples + kBlock * per - 1) / (kBlock * per)), (unsigned)n);
  if (per4)
    hipLaunchKernelGGL(k_megb_prep<kPassPer>, grid, dim3(kBlock), 0, stream, b.sample_off, total_samples,
                       max_samples, poses, mask, rec, quat, trans);
  else
    hipLaunchKernelGGL(k_megb_prep<1>, grid, dim3(kBlock), 0, stream, b.sample_off, total_samples, max_samples,
                       poses, mask, rec, quat, trans);
  // The wide variant while there are at most as many chains as compute
  // units, else the narrow one (measured on batches of 256-1,024 uneven
  // instances: 1.4-2.3 times faster than the shell steps of one wave with no
  // pipelined segments, which ran at the same four chains per compute unit).
  // The variants keep shells of different capacities, which the first-phase
  // kernel must know.
  int dev = 0, n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    n_cu = 0;
  const bool wide = 2 * n <= n_cu;
  const int cap = wide ? chain_cap<kChainWide>() : chain_cap<kChainNarrow>();
  const size_t lds = (size_t)cap * (sizeof(float4) + sizeof(int));
  const int no_prune = (p.flags & PURSE_FLAG_NO_PRUNING) ? 1 : 0;
  const int64_t gstride = gshell_stride(total_samples, max_samples);
  if (early_phase_applies(max_samples, p.megb_iters, p.megb_avg, no_prune)) {
    const dim3 eg((unsigned)kEarlyWG, 2u, (unsigned)n);
    for (int i = 1; i <= kEarlySteps + 1; ++i)
      hipLaunchKernelGGL(k_megb_early, eg, dim3(kEarlyBlock), 0, stream, b.sample_off, total_samples, max_samples,
                         quat, trans, rec, es, dref, trace, ckpt, ck, p.megb_iters, p.megb_avg, cap, no_prune, i);
    hipLaunchKernelGGL(k_megb_gshell_hist, eg, dim3(kEarlyBlock), 0, stream, b.sample_off, total_samples,
                       max_samples, rec, es, dref, p.megb_iters, p.megb_avg, cap, no_prune);
    hipLaunchKernelGGL(k_megb_gshell_collect, eg, dim3(kEarlyBlock), 0, stream, b.sample_off, total_samples,
                       max_samples, quat, trans, rec, es, dref, gid, gpt, gstride, p.megb_iters, p.megb_avg, cap,
                       no_prune);
  }
  if (wide)
    hipLaunchKernelGGL(k_megb_chain<kChainWide>, dim3(2 * n), dim3(chain_block<kChainWide>()), lds, stream,
                       b.sample_off, max_samples, quat, trans, rec, dref, total_samples, trace, ckpt, ck, p.megb_iters,
                       p.megb_avg, cap, no_prune, gid, gpt, gstride);
  else
    hipLaunchKernelGGL(k_megb_chain<kChainNarrow>, dim3(2 * n), dim3(chain_block<kChainNarrow>()), lds, stream,
                       b.sample_off, max_samples, quat, trans, rec, dref, total_samples, trace, ckpt, ck, p.megb_iters,
                       p.megb_avg, cap, no_prune, gid, gpt, gstride);
  hipLaunchKernelGGL(k_megb_sign, dim3(n), dim3(kBlock), 0, stream, b.sample_off, total_samples, max_samples, poses,
                     trace, rec, p.megb_iters, ck);
  if (p.flags & PURSE_FLAG_EXACT_MEB)
    hipLaunchKernelGGL(k_megb_exact, dim3(2 * n), dim3(kBlock), 0, stream, b.sample_off, total_samples, max_samples,
                       quat, trans, rec);
  if (per4)
    hipLaunchKernelGGL(k_megb_radii<kPassPer>, grid, dim3(kBlock), 0, stream, b.sample_off, total_samples,
                       max_samples, poses, mask, rec);
  else
    hipLaunchKernelGGL(k_megb_radii<1>, grid, dim3(kBlock), 0, stream, b.sample_off, total_samples, max_samples,
                       poses, mask, rec);
  hipLaunchKernelGGL(k_megb_final, dim3((n + 255) / 256), dim3(256), 0, stream, n, rec, centre, radii,
                     n_feasible, inst_status);
}

}  // namespace purse
