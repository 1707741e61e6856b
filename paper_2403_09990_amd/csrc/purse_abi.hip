// Host side of the C ABI: argument validation, workspace carving, launches.
// Nothing here allocates device memory or synchronises the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "purse_launch.hpp"

namespace {

thread_local std::string g_last_error;

purse_status fail(purse_status s, const char *msg) {
  g_last_error = msg;
  return s;
}

purse_status hip_check(hipError_t e, const char *where) {
  if (e == hipSuccess) return PURSE_OK;
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return PURSE_E_HIP;
}

purse_status check_device() {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    g_last_error = "no HIP device";
    return PURSE_E_NO_DEVICE;
  }
  return PURSE_OK;
}

purse_status check_batch(const purse_batch *b) {
  if (!b) return fail(PURSE_E_NULL, "batch is NULL");
  if (!b->kind || !b->n_kp || !b->kp_off || !b->sample_off || !b->model_pts || !b->centres || !b->shapes ||
      !b->bounds || !b->intrinsics || !b->seed)
    return fail(PURSE_E_NULL, "a batch array is NULL");
  if (b->n_inst < 1 || b->n_inst > 65535) return fail(PURSE_E_BAD_ARG, "n_inst must be in [1, 65535]");
  if (b->max_kp < 3 || b->max_kp > PURSE_MAX_KP) return fail(PURSE_E_BAD_ARG, "max_kp must be in [3, 64]");
  if (b->total_kp < 3 || b->total_kp > (int64_t)b->n_inst * PURSE_MAX_KP)
    return fail(PURSE_E_BAD_ARG, "total_kp out of range");
  if (b->total_samples < 1 || b->max_samples < 1 || b->max_samples > b->total_samples ||
      b->max_samples > (int64_t)INT32_MAX - 1024)
    return fail(PURSE_E_BAD_ARG, "sample counts out of range");
  return PURSE_OK;
}

purse_status check_params(const purse_params *p) {
  if (!p) return fail(PURSE_E_NULL, "params is NULL");
  if (p->n_iters < 0 || p->n_iters > 100000) return fail(PURSE_E_BAD_ARG, "n_iters out of range");
  if (p->n_gn < 1 || p->n_gn > 64) return fail(PURSE_E_BAD_ARG, "n_gn out of range");
  if (p->n_bis < 0 || p->n_bis > 30) return fail(PURSE_E_BAD_ARG, "n_bis out of range");
  if (p->megb_iters < 1 || p->megb_iters > (1 << 24)) return fail(PURSE_E_BAD_ARG, "megb_iters out of range");
  if (p->megb_avg < 1 || p->megb_avg > p->megb_iters) return fail(PURSE_E_BAD_ARG, "megb_avg out of range");
  if (!(p->kappa > 0.f && p->kappa <= 1.f)) return fail(PURSE_E_BAD_ARG, "kappa must be in (0, 1]");
  if (!(p->tau_abs_3d >= 0.f) || !(p->tau_abs_2d >= 0.f)) return fail(PURSE_E_BAD_ARG, "tau must be >= 0");
  if (!(p->z_min > 0.f)) return fail(PURSE_E_BAD_ARG, "z_min must be > 0");
  if (!(p->omega0 >= 0.f && p->omega0 < 3.f) || !(p->v0 >= 0.f) || !std::isfinite(p->v0))
    return fail(PURSE_E_BAD_ARG, "omega0 / v0 out of range");
  if (p->ckpt_every < 1) return fail(PURSE_E_BAD_ARG, "ckpt_every must be >= 1");
  if (p->centre_gn < 1 || p->centre_gn > 100) return fail(PURSE_E_BAD_ARG, "centre_gn out of range");
  if (!(p->tile == 0 || p->tile == 64 || p->tile == 128 || p->tile == 256))
    return fail(PURSE_E_BAD_ARG, "tile must be 0, 64, 128 or 256");
  if (p->waves_per_simd < 0 || p->waves_per_simd > 8) return fail(PURSE_E_BAD_ARG, "waves_per_simd must be 0..8");
  return PURSE_OK;
}

purse::DevBatch dev_batch(const purse_batch *b) {
  purse::DevBatch d;
  d.n_inst = b->n_inst;
  d.max_kp = b->max_kp;
  d.total_kp = b->total_kp;
  d.total_samples = b->total_samples;
  d.max_samples = b->max_samples;
  d.kind = b->kind;
  d.n_kp = b->n_kp;
  d.kp_off = b->kp_off;
  d.sample_off = b->sample_off;
  d.model_pts = b->model_pts;
  d.centres = b->centres;
  d.shapes = b->shapes;
  d.bounds = b->bounds;
  d.intrinsics = b->intrinsics;
  d.seed = b->seed;
  return d;
}

purse::DevParams dev_params(const purse_params *p) {
  purse::DevParams d;
  d.n_iters = p->n_iters;
  d.n_gn = p->n_gn;
  d.n_bis = p->n_bis;
  d.megb_iters = p->megb_iters;
  d.megb_avg = p->megb_avg;
  d.centre_gn = p->centre_gn;
  d.ckpt_every = p->ckpt_every;
  d.flags = p->flags;
  d.omega0 = p->omega0;
  d.v0 = p->v0;
  d.kappa = p->kappa;
  d.tau3 = p->tau_abs_3d;
  d.tau2 = p->tau_abs_2d;
  d.z_min = p->z_min;
  return d;
}

purse::WsLayout layout_for(const purse_batch *b, const purse_params *p) {
  return purse::ws_layout(b->n_inst, b->total_kp, b->total_samples, b->max_samples, b->max_kp, p->megb_iters,
                          p->ckpt_every);
}

purse_status check_ws(const purse_batch *b, const purse_params *p, void *ws, size_t ws_bytes) {
  if (!ws) return fail(PURSE_E_NULL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % purse::kAlign) return fail(PURSE_E_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < layout_for(b, p).total) return fail(PURSE_E_WORKSPACE, "workspace too small");
  return PURSE_OK;
}

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// The sampler's part of a call: prologue (unless reused) and trajectories,
// with the instance records, keypoint records and tile schedule in ws (the
// first three regions of the workspace layout).
purse_status sample_into(const purse_batch *b, const purse_params *p, float *poses, uint8_t *mask,
                         int32_t *inst_status, void *ws, hipStream_t st) {
  const purse::WsLayout L = layout_for(b, p);
  const purse::DevBatch db = dev_batch(b);
  const purse::DevParams dp = dev_params(p);
  auto *inst = at<purse::InstRec>(ws, L.inst);
  auto *kp = at<purse::KpRec>(ws, L.kp);
  purse_status s;
  if (!(p->flags & PURSE_FLAG_REUSE_PROLOGUE)) {
    purse::launch_prologue(db, dp, inst, kp, inst_status, st);
    if ((s = hip_check(hipGetLastError(), "prologue launch"))) return s;
  }
  const int tile = p->tile ? p->tile : 256;
  if (purse::sample_grid(b->total_samples, b->n_inst, tile / 2) > INT32_MAX)
    return fail(PURSE_E_BAD_ARG, "too many sample tiles for one launch");
  const hipError_t e = purse::launch_sample(db, dp, inst, kp, at<int32_t>(ws, L.sched), poses, mask, tile,
                                            b->total_samples, p->waves_per_simd, st);
  if (e != hipSuccess) return hip_check(e, "sampler stream join");
  return hip_check(hipGetLastError(), "sampler launch");
}

// ---------------------------------------------------------------------------
// Static scratch of purse_sample_noalloc: room for the instance records,
// keypoint records and tile schedule of a batch of at most kNoAllocMaxInst
// instances and kNoAllocMaxKp keypoints (3.4 MB), held by every device the
// library runs on until the process ends.  In host code `scratch` names a
// host-side stand-in; the device address comes from hipGetSymbolAddress, once
// per device, and only that address is ever passed to a kernel.
constexpr int64_t kNoAllocMaxInst = 1024;
constexpr int64_t kNoAllocMaxKp = 65536;
constexpr size_t kScratchBytes =
    purse::align_up(sizeof(purse::InstRec) * kNoAllocMaxInst) + purse::align_up(sizeof(purse::KpRec) * kNoAllocMaxKp) +
    purse::align_up(sizeof(int32_t) * purse::kSchedGroups * (2 * kNoAllocMaxInst + 2));

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of the current device's scratch array (looked up on the
// first call on that device, with the device current).
purse_status scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(PURSE_E_NO_DEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % purse::kAlign)
      return fail(PURSE_E_HIP, "static scratch has no aligned device address");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return PURSE_OK;
}

}  // namespace

extern "C" {

purse_status purse_default_params(purse_params *p) {
  if (!p) return fail(PURSE_E_NULL, "params is NULL");
  p->n_iters = 50;
  p->n_gn = 2;
  p->n_bis = 16;
  p->megb_iters = 4096;
  p->megb_avg = 10;
  p->omega0 = 0.5f;
  p->v0 = 0.2f;
  p->kappa = 0.999f;
  p->tau_abs_3d = 1e-5f;
  p->tau_abs_2d = 1e-4f;
  p->z_min = 1e-3f;
  p->ckpt_every = 5;
  p->centre_gn = 50;
  p->tile = 0;
  p->flags = 0;
  p->waves_per_simd = 0;
  return PURSE_OK;
}

purse_status purse_workspace_size(const purse_batch *b, const purse_params *p, size_t *bytes) {
  if (!bytes) return fail(PURSE_E_NULL, "bytes is NULL");
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  *bytes = layout_for(b, p).total;
  return PURSE_OK;
}

purse_status purse_sample(const purse_batch *b, const purse_params *p, float *poses, uint8_t *mask,
                          int32_t *inst_status, void *ws, size_t ws_bytes, void *stream) {
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  if (!poses || !mask || !inst_status) return fail(PURSE_E_NULL, "an output is NULL");
  if ((s = check_ws(b, p, ws, ws_bytes))) return s;
  if ((s = check_device())) return s;
  return sample_into(b, p, poses, mask, inst_status, ws, static_cast<hipStream_t>(stream));
}

purse_status purse_sample_noalloc(const purse_batch *b, const purse_params *p, float *poses, uint8_t *mask,
                                  int32_t *inst_status, void *stream) {
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  if (!poses || !mask || !inst_status) return fail(PURSE_E_NULL, "an output is NULL");
  if (b->n_inst > kNoAllocMaxInst || b->total_kp > kNoAllocMaxKp)
    return fail(PURSE_E_BAD_ARG, "batch beyond the static scratch (at most 1024 instances, 65536 keypoints)");
  if (layout_for(b, p).megb > kScratchBytes)
    return fail(PURSE_E_BAD_ARG, "batch beyond the static scratch");
  if ((s = check_device())) return s;
  void *ws = nullptr;
  if ((s = scratch_address(&ws))) return s;
  return sample_into(b, p, poses, mask, inst_status, ws, static_cast<hipStream_t>(stream));
}

purse_status purse_megb(const purse_batch *b, const purse_params *p, const float *poses, const uint8_t *mask,
                        float *centre, double *radii, int64_t *n_feasible, int32_t *trace, int32_t *inst_status,
                        void *ws, size_t ws_bytes, void *stream) {
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  if (!poses || !mask || !centre || !radii || !n_feasible || !trace || !inst_status)
    return fail(PURSE_E_NULL, "an argument is NULL");
  if ((s = check_ws(b, p, ws, ws_bytes))) return s;
  if ((s = check_device())) return s;
  const purse::WsLayout L = layout_for(b, p);
  const purse::DevBatch db = dev_batch(b);
  const purse::DevParams dp = dev_params(p);
  purse::launch_megb(db, dp, poses, mask, at<purse::MegbRec>(ws, L.megb), at<float4>(ws, L.quat),
                     at<float4>(ws, L.trans), at<float>(ws, L.dref), at<float4>(ws, L.ckpt),
                     at<purse::EarlyScratch>(ws, L.early), at<int32_t>(ws, L.gid), at<float4>(ws, L.gpt), centre,
                     radii, n_feasible, trace, inst_status, b->max_samples, b->total_samples,
                     static_cast<hipStream_t>(stream));
  return hip_check(hipGetLastError(), "megb launch");
}

purse_status purse_megb_backward(const purse_batch *b, const purse_params *p, const float *poses,
                                 const uint8_t *mask, const int32_t *trace, const double *g_radii,
                                 const float *g_centre, float *g_centres, float *g_shapes, float *g_bounds,
                                 int32_t *bwd_status, void *ws, size_t ws_bytes, void *stream) {
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  if (!poses || !mask || !trace || !g_radii || !g_centre || !g_centres || !g_shapes || !g_bounds)
    return fail(PURSE_E_NULL, "an argument is NULL");
  if (p->flags & PURSE_FLAG_EXACT_MEB)
    return fail(PURSE_E_BAD_ARG, "the backward differentiates the descent's centre, not the exact ball");
  if ((s = check_ws(b, p, ws, ws_bytes))) return s;
  if ((s = check_device())) return s;
  const purse::WsLayout L = layout_for(b, p);
  const purse::DevBatch db = dev_batch(b);
  const purse::DevParams dp = dev_params(p);
  const hipError_t e = purse::launch_backward(db, dp, poses, mask, trace, g_radii, g_centre, at<purse::InstRec>(ws, L.inst),
                         at<purse::KpRec>(ws, L.kp), at<purse::MegbRec>(ws, L.megb), at<purse::BwdRec>(ws, L.bwd),
                         at<float4>(ws, L.ckpt), at<float>(ws, L.tan), at<float>(ws, L.contrib),
                         at<int64_t>(ws, L.items), g_centres, g_shapes, g_bounds, bwd_status,
                         static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_check(e, "backward stream join");
  return hip_check(hipGetLastError(), "backward launch");
}

purse_status purse_init(const purse_batch *b, const purse_params *p, float *poses, uint8_t *mask, void *stream) {
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  if (!poses || !mask) return fail(PURSE_E_NULL, "an output is NULL");
  if ((s = check_device())) return s;
  purse::launch_init(dev_batch(b), dev_params(p), poses, mask, static_cast<hipStream_t>(stream));
  return hip_check(hipGetLastError(), "init launch");
}

purse_status purse_walk_default_params(purse_walk_params *w) {
  if (!w) return fail(PURSE_E_NULL, "walk params is NULL");
  w->n_walks = 2;
  w->n_iters = 5;
  w->n_perturb = 150;
  w->n_keep = 10;
  w->n_scales = 15;
  w->gamma = 0.5f;
  w->omega0 = 0.5f;
  w->v0 = 0.05f;
  w->t_pert = 0.005f;
  w->r_pert = 0.02f;
  return PURSE_OK;
}

purse_status purse_walk_workspace_size(const purse_batch *b, size_t *bytes) {
  if (!bytes) return fail(PURSE_E_NULL, "bytes is NULL");
  purse_status s = check_batch(b);
  if (s) return s;
  *bytes = purse::align_up(sizeof(float) * 12 * (size_t)b->n_inst);
  return PURSE_OK;
}

purse_status purse_walk(const purse_batch *b, const purse_params *p, const purse_walk_params *w,
                        const int64_t *start_off, const float *starts, int64_t total_starts, float *poses,
                        uint8_t *mask, int32_t *decisions, void *ws, size_t ws_bytes, void *stream) {
  purse_status s = check_batch(b);
  if (s) return s;
  if ((s = check_params(p))) return s;
  if (!w) return fail(PURSE_E_NULL, "walk params is NULL");
  if (w->n_walks < 1 || w->n_walks > 1 << 20 || w->n_iters < 0 || w->n_iters > 10000 || w->n_perturb < 1 ||
      w->n_perturb > purse::kWalkMaxPerturb || w->n_keep < 1 || w->n_keep > purse::kWalkMaxKeep ||
      w->n_keep > w->n_perturb || w->n_scales < 1 || w->n_scales > purse::kWalkMaxScales)
    return fail(PURSE_E_BAD_ARG, "walk counts out of range (N_P <= 256, N_P* <= min(16, N_P), N_T <= 32)");
  if (!(w->gamma > 0.f && w->gamma <= 1.f) || !(w->omega0 >= 0.f && w->omega0 < 3.f) || !(w->v0 >= 0.f) ||
      !std::isfinite(w->v0) || !(w->t_pert >= 0.f) || !std::isfinite(w->t_pert) || !(w->r_pert >= 0.f) ||
      !(w->r_pert < 3.f))
    return fail(PURSE_E_BAD_ARG, "walk scales out of range");
  if (total_starts < 0 || total_starts > ((int64_t)1 << 40) / w->n_walks)
    return fail(PURSE_E_BAD_ARG, "total_starts out of range");
  if (!start_off || !starts || !poses || !mask) return fail(PURSE_E_NULL, "an argument is NULL");
  if (!ws) return fail(PURSE_E_NULL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % purse::kAlign) return fail(PURSE_E_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < purse::align_up(sizeof(float) * 12 * (size_t)b->n_inst)) return fail(PURSE_E_WORKSPACE, "workspace too small");
  if ((s = check_device())) return s;
  purse::WalkParams wp;
  wp.n_walks = w->n_walks;
  wp.n_iters = w->n_iters;
  wp.n_perturb = w->n_perturb;
  wp.n_keep = w->n_keep;
  wp.n_scales = w->n_scales;
  wp.gamma = w->gamma;
  wp.omega0 = w->omega0;
  wp.v0 = w->v0;
  wp.t_pert = w->t_pert;
  wp.r_pert = w->r_pert;
  purse::launch_walk(dev_batch(b), dev_params(p), wp, start_off, total_starts, starts, static_cast<float *>(ws), poses,
                     mask, decisions, static_cast<hipStream_t>(stream));
  return hip_check(hipGetLastError(), "walk launch");
}

const char *purse_status_string(purse_status s) {
  switch (s) {
    case PURSE_OK: return "ok";
    case PURSE_E_NULL: return "a required pointer is NULL";
    case PURSE_E_BAD_ARG: return "argument out of range";
    case PURSE_E_WORKSPACE: return "workspace too small or misaligned";
    case PURSE_E_NO_DEVICE: return "no usable HIP device";
    case PURSE_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *purse_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
