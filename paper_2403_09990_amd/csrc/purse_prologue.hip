// Per-instance prologue: validation, keypoint records, centre fit (float64),
// pivot and feasible anchor.  Two wavefronts per instance: validation and the
// keypoint records take one keypoint per lane of wavefront 0; the 2D-3D
// centre fit is a float64 Gauss-Newton iteration from two starts, one start
// per wavefront (formed by lane 0, iterated with one keypoint per lane), so
// the two run on different SIMDs at once; the rest (Arun's fit, the pivot,
// the anchor) is serial in lane 0 of wavefront 0.
#include "purse_bwd_check.hpp"
#include "purse_fit.hpp"
#include "purse_launch.hpp"
#include "purse_traj.hpp"

namespace purse {

constexpr int kPrologueBlock = 128;

__global__ void __launch_bounds__(kPrologueBlock) k_prologue(DevBatch b, DevParams p, InstRec *inst, KpRec *kprec,
                                                             int32_t *inst_status) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double w_s[3 * PURSE_MAX_KP];  // whitening factors of the keypoints
  __shared__ double fit_R[2][9], fit_t[2][3], fit_cost[2];
  __shared__ int fit_good[2], stage;         // stage: 0 invalid, 1 valid 3D-3D, 2 valid 2D-3D
  __shared__ int fp_n;                       // keypoints the data fingerprint covers
  __shared__ int64_t fp_ko;
  InstRec I;                                 // (lane 0 of wavefront 0)
  double ab[3] = {0, 0, 0};
  if (tid < 64) {
    // ---- header: every lane of wavefront 0 reads it, lane 0 keeps the record
    const int kind = b.kind[j];
    const int n = b.n_kp[j];
    const int64_t kp_off = b.kp_off[j];
    int64_t soff, sM;
    sample_range(b.sample_off, j, b.total_samples, b.max_samples, soff, sM);
    const bool kp_ok = kp_off >= 0 && b.kp_off[j + 1] - kp_off == (int64_t)n && b.kp_off[j + 1] <= b.total_kp;
    const bool is2d = kind == PURSE_KIND_2D3D;
    const int64_t ko = kp_ok ? kp_off : 0;
    float K[4];
    for (int k = 0; k < 4; ++k) K[k] = is2d ? b.intrinsics[4 * j + k] : 0.f;
    const float *a = b.model_pts + 3 * ko;
    const float *c = b.centres + 3 * ko;
    const float *L = b.shapes + 4 * ko;
    const float *beta = b.bounds + ko;
    int status = PURSE_INST_OK;
    // ---- validation: keypoint i on lane i (at most PURSE_MAX_KP = 64)
    if ((kind != PURSE_KIND_3D3D && !is2d) || !kp_ok || n < (is2d ? 6 : 3) || n > PURSE_MAX_KP || sM < 1 ||
        n > b.max_kp) {
      status = PURSE_INST_BAD_SIZE;
    } else {
      bool good = true;
      if (tid < n) {
        const int i = tid;
        for (int r = 0; r < 3; ++r) good = good && finite_f(a[3 * i + r]);
        good = good && finite_f(c[3 * i]) && finite_f(c[3 * i + 1]) && (is2d || finite_f(c[3 * i + 2]));
        good = good && finite_f(beta[i]) && beta[i] >= 0.f;
        if (is2d) {
          const float *l = L + 4 * i;
          good = good && finite_f(l[0]) && finite_f(l[1]) && finite_f(l[2]) && finite_f(l[3]);
          good = good && l[1] == l[2] && l[0] > 0.f && (double)l[0] * l[3] - (double)l[1] * l[2] > 0.0;
        }
      }
      if (is2d)
        for (int k = 0; k < 4; ++k) good = good && finite_f(K[k]);
      if (is2d) good = good && K[0] > 0.f && K[1] > 0.f;
      if (__ballot(!good) != 0ull) status = PURSE_INST_BAD_SHAPE;
    }
    if (status == PURSE_INST_OK) {
      // ---- model centroid (a sum over the lanes in a fixed butterfly order)
      // and the record of keypoint `tid` (with the whitening factors of the fit)
      for (int r = 0; r < 3; ++r) ab[r] = tid < n ? (double)a[3 * tid + r] : 0.0;
      for (int o = 32; o >= 1; o >>= 1)
        for (int r = 0; r < 3; ++r) ab[r] += __shfl_xor(ab[r], o, 64);
      for (int r = 0; r < 3; ++r) ab[r] /= n;
      const float tau = is2d ? p.tau2 : p.tau3;
      if (tid < n) {
        const int i = tid;
        KpRec k;
        for (int r = 0; r < 3; ++r) {
          k.m[r] = is2d ? a[3 * i + r] : (float)((double)a[3 * i + r] - ab[r]);
          k.c[r] = (r < 2 || !is2d) ? c[3 * i + r] : 0.f;
          k.w[r] = 0.f;
        }
        if (is2d) {
          double *w = w_s + 3 * i;
          whiten_factor<double>(L + 4 * i, w);
          for (int r = 0; r < 3; ++r) k.w[r] = (float)w[r];
        }
        k.kb = (float)((double)p.kappa * beta[i]);
        k.kb2 = k.kb * k.kb;
        k.bt = (float)((double)beta[i] + tau);
        kprec[kp_off + i] = k;
      }
    }
    if (tid == 0) {
      I.kind = kind;
      I.n_kp = n;
      I.kp_off = kp_off;
      I.sample_off = soff;
      I.n_samples = sM;
      I.seed = b.seed[j];
      I.has_anchor = 0;
      I.status = status;
      for (int k = 0; k < 4; ++k) I.K[k] = K[k];
      for (int k = 0; k < 9; ++k) I.Rc[k] = I.Ra[k] = (k % 4 == 0) ? 1.f : 0.f;
      for (int k = 0; k < 3; ++k) I.tc[k] = I.ta[k] = I.oc[k] = 0.f;
      for (int r = 0; r < 3; ++r) I.abar[r] = status == PURSE_INST_OK ? (float)ab[r] : 0.f;
      I.data_fp = 0ull;
      fp_n = (kp_ok && n >= 0 && n <= PURSE_MAX_KP) ? n : 0;
      fp_ko = ko;
      stage = status != PURSE_INST_OK ? 0 : (is2d ? 2 : 1);
    }
  }
  __syncthreads();
  const int st = stage;
  // fingerprint of the instance's inputs (one keypoint per lane of
  // wavefront 0), which the backward compares with the batch it is given
  if (tid < 64) {
    unsigned long long h = 0ull;
    if (tid < fp_n) {
      const int64_t k = fp_ko + tid;
      uint32_t w[11];
      kp_words(b.kind[j], b.model_pts + 3 * k, b.centres + 3 * k, b.shapes + 4 * k, b.bounds[k], w);
      h = kp_data_term(tid, w);
    }
    for (int o = 32; o >= 1; o >>= 1) h += __shfl_xor(h, o, 64);
    if (tid == 0) I.data_fp = h + (I.kind == PURSE_KIND_2D3D ? intrinsics_term(I.K) : 0ull);
  }
  if (st == 2) {
    // Gauss-Newton from the DLT (wavefront 0) and from the weak-perspective
    // fit (wavefront 1): lane 0 forms the start, the whole wavefront iterates
    const int f = tid >> 6;
    const int n = b.n_kp[j];
    const int64_t ko = b.kp_off[j];
    const float *a = b.model_pts + 3 * ko, *c = b.centres + 3 * ko;
    const float K[4] = {b.intrinsics[4 * j], b.intrinsics[4 * j + 1], b.intrinsics[4 * j + 2], b.intrinsics[4 * j + 3]};
    const ObsCached obs{c, w_s};
    if ((tid & 63) == 0) {
      double R[9], t[3];
      const bool ok = f == 0 ? dlt_2d(a, c, n, K, R, t) : affine_2d(a, c, n, K, R, t);
      fit_good[f] = ok;
      for (int k = 0; k < 9; ++k) fit_R[f][k] = R[k];
      for (int k = 0; k < 3; ++k) fit_t[f][k] = t[k];
    }
    __syncthreads();
    bool ok = fit_good[f] != 0;
    double R[9], t[3];
    for (int k = 0; k < 9; ++k) R[k] = fit_R[f][k];
    for (int k = 0; k < 3; ++k) t[k] = fit_t[f][k];
    __syncthreads();
    if (ok) ok = gn_centre_2d_wave(a, obs, n, K, p.centre_gn, (double)p.z_min, R, t);
    if ((tid & 63) == 0) {
      fit_good[f] = ok;
      if (ok) {
        for (int k = 0; k < 9; ++k) fit_R[f][k] = R[k];
        for (int k = 0; k < 3; ++k) fit_t[f][k] = t[k];
        fit_cost[f] = cost_2d_obs(a, obs, n, K, R, t);
      }
    }
  }
  __syncthreads();
  if (tid != 0) return;
  if (st == 0) {
    inst[j] = I;
    inst_status[j] = I.status;
    return;
  }
  const int n = I.n_kp;
  const bool is2d = st == 2;
  const float *a = b.model_pts + 3 * I.kp_off;
  const float *c = b.centres + 3 * I.kp_off;
  KpRec *kp = kprec + I.kp_off;
  // ---- centre fit: the successful fit with the lower cost (ties: the DLT one)
  double Rd[9], td[3];
  bool fit_ok = true;
  if (is2d) {
    const bool ok1 = fit_good[0] != 0, ok2 = fit_good[1] != 0;
    const int f = (ok2 && (!ok1 || fit_cost[1] < fit_cost[0])) ? 1 : 0;
    fit_ok = ok1 || ok2;
    for (int k = 0; k < 9; ++k) Rd[k] = fit_ok ? fit_R[f][k] : (k % 4 == 0 ? 1.0 : 0.0);
    for (int k = 0; k < 3; ++k) td[k] = fit_ok ? fit_t[f][k] : 0.0;
  } else {
    kabsch_centre(a, c, n, Rd, td);
  }
  for (int k = 0; k < 9; ++k) I.Rc[k] = (float)Rd[k];
  for (int r = 0; r < 3; ++r) I.tc[r] = (float)td[r];
  if (!fit_ok) {
    I.status = PURSE_INST_FIT_FAILED;
    inst[j] = I;
    inst_status[j] = I.status;
    return;
  }
  double oc[3];
  matvec3(Rd, ab, oc);
  for (int r = 0; r < 3; ++r) I.oc[r] = (float)(oc[r] + td[r]);
  // ---- anchor: x_c if inside the kappa-shrunk set, else the end of one
  // trajectory from x_c with no offset if that one is
  Pose xc;
  for (int k = 0; k < 9; ++k) xc.R[k] = I.Rc[k];
  for (int r = 0; r < 3; ++r) xc.t[r] = I.tc[r];
  const KpPlain kpl{kp};
  bool inside = is2d ? feasible<PURSE_KIND_2D3D>(I, kpl, xc, p, p.kappa)
                     : feasible<PURSE_KIND_3D3D>(I, kpl, xc, p, p.kappa);
  if (inside) {
    I.has_anchor = 1;
    for (int k = 0; k < 9; ++k) I.Ra[k] = xc.R[k];
    for (int r = 0; r < 3; ++r) I.ta[r] = xc.t[r];
  } else {
    I.status |= PURSE_INST_ANCHOR_ITERATED;
    int nfb = 0;
    Pose x = xc;
    const FrameT<float> F = frame_of<float>(I);
    uint8_t m = is2d ? run_trajectory<PURSE_KIND_2D3D>(I, F, kpl, x, p, false, nfb)
                     : run_trajectory<PURSE_KIND_3D3D>(I, F, kpl, x, p, false, nfb);
    bool ok = (m & PURSE_MASK_FAILED) == 0;
    if (ok)
      ok = is2d ? feasible<PURSE_KIND_2D3D>(I, kpl, x, p, p.kappa) : feasible<PURSE_KIND_3D3D>(I, kpl, x, p, p.kappa);
    if (ok) {
      I.has_anchor = 1;
      for (int k = 0; k < 9; ++k) I.Ra[k] = x.R[k];
      for (int r = 0; r < 3; ++r) I.ta[r] = x.t[r];
    } else {
      I.status |= PURSE_INST_NO_ANCHOR;
    }
  }
  inst[j] = I;
  inst_status[j] = I.status;
}

void launch_prologue(const DevBatch &b, const DevParams &p, InstRec *inst, KpRec *kp, int32_t *inst_status,
                     hipStream_t stream) {
  hipLaunchKernelGGL(k_prologue, dim3(b.n_inst), dim3(kPrologueBlock), 0, stream, b, p, inst, kp, inst_status);
}

}  // namespace purse
