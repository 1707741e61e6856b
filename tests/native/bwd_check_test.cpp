// Host-side exercise of the backward's index guards (purse_bwd_check.hpp) at
// the shapes of the 64 x 2^20 and 512-instance workloads, with adversarial
// inputs: instance records of another instance or of random bytes, trace
// entries outside the instance or infeasible, more distinct winners than the
// active set holds, and a non-finite centre.  The driver below re-enacts the
// backward's per-instance index path (first feasible sample, trace check,
// active set, radius argmax in the kernel's thread order, insertion) with the
// same functions the kernels call, collects every global index the kernel
// would then form (poses, mask, checkpoints, tangents, contributions,
// keypoint records) and checks that each lies inside its array, or that the
// instance was stopped with an error status before any was formed.
//
// It also shows the mechanism the guards close: without the status check, a
// non-finite centre leaves the radius argmax at its sentinel INT32_MAX, which
// the active set then takes as a sample id, and the pose index formed from it
// lies about 100 GB past the poses array.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>

#include "../../paper_2403_09990_amd/csrc/purse_bwd_check.hpp"

using namespace purse;

static int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                           \
    }                                                                     \
  } while (0)

struct Rng {
  unsigned long long s;
  unsigned long long next() { return s = mix64(s); }
  double unit() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Batch arrays (host copies of what the kernels read).
struct HostBatch {
  int n;
  std::vector<int32_t> kind, n_kp;
  std::vector<int64_t> kp_off, sample_off;
  std::vector<uint64_t> seed;
  int64_t total_kp, total_samples, max_samples;
  int max_kp;
  InstView view(int j) const {
    InstView v;
    v.kind = kind[j];
    v.n_kp = n_kp[j];
    v.kp_off = kp_off[j];
    v.kp_end = kp_off[j + 1];
    v.s_off = sample_off[j];
    v.s_end = sample_off[j + 1];
    v.seed = seed[j];
    v.total_kp = total_kp;
    v.total_samples = total_samples;
    v.max_samples = max_samples;
    return v;
  }
};

static HostBatch make_batch(const std::vector<int> &kinds, const std::vector<int> &nkp, const std::vector<int64_t> &ms) {
  HostBatch b;
  b.n = (int)kinds.size();
  b.kind.assign(kinds.begin(), kinds.end());
  b.n_kp.assign(nkp.begin(), nkp.end());
  b.kp_off.assign(b.n + 1, 0);
  b.sample_off.assign(b.n + 1, 0);
  b.seed.resize(b.n);
  b.max_samples = 0;
  b.max_kp = 0;
  for (int j = 0; j < b.n; ++j) {
    b.kp_off[j + 1] = b.kp_off[j] + nkp[j];
    b.sample_off[j + 1] = b.sample_off[j] + ms[j];
    b.seed[j] = 1000 + j;
    if (ms[j] > b.max_samples) b.max_samples = ms[j];
    if (nkp[j] > b.max_kp) b.max_kp = nkp[j];
  }
  b.total_kp = b.kp_off[b.n];
  b.total_samples = b.sample_off[b.n];
  return b;
}

// The record the prologue writes for instance j.
static InstRec record_of(const HostBatch &b, int j) {
  InstRec I;
  std::memset(&I, 0, sizeof I);
  I.kind = b.kind[j];
  I.n_kp = b.n_kp[j];
  I.kp_off = b.kp_off[j];
  I.sample_off = b.sample_off[j];
  I.n_samples = b.sample_off[j + 1] - b.sample_off[j];
  I.seed = b.seed[j];
  return I;
}

// Rotation entries of sample s (a deterministic rotation per id) and whether
// it is feasible.
static void sample_rot(uint64_t key, int s, double R[9]) {
  Rng r{key * 0x9E37ull + (unsigned long long)s};
  double q[4];
  double n2 = 0;
  for (int k = 0; k < 4; ++k) {
    q[k] = r.unit() - 0.5;
    n2 += q[k] * q[k];
  }
  const double n = 1.0 / std::sqrt(n2);
  const double w = q[0] * n, x = q[1] * n, y = q[2] * n, z = q[3] * n;
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
static bool feasible_of(uint64_t key, int s) { return (mix64(key ^ (unsigned long long)s) & 7u) != 0u; }

struct Outcome {
  int32_t status;
  int n_act;
  bool indices_ok;
  long long n_indices;
};

constexpr int kBlock = 256;  // the backward's workgroup size

// The backward's index path for instance j; `trace` holds T (rotation,
// translation) winner pairs; `Rstar` may be non-finite.  When `unguarded`,
// the radius samples are inserted without the status checks (the code before
// the guards), and the first out-of-range index is reported.
static Outcome run_instance(const HostBatch &b, int j, const InstRec &I, const std::vector<int> &trace, int T,
                            int avg, int ck, const double Rstar[9], bool unguarded, int64_t *bad_index) {
  Outcome o{kBwdOk, 0, true, 0};
  const int64_t poses_words = 12 * b.total_samples;
  auto need = [&](int64_t idx, int64_t size) {
    ++o.n_indices;
    if (idx < 0 || idx >= size) {
      o.indices_ok = false;
      if (bad_index && *bad_index < 0) *bad_index = idx;
    }
  };
  const InstView v = b.view(j);
  if (!inst_record_ok(I, v)) {
    o.status = kBwdStale;
    return o;
  }
  const int64_t off = v.s_off;
  const int M = (int)(v.s_end - v.s_off);
  const uint64_t key = v.seed;
  // first feasible sample
  int s0 = INT32_MAX;
  for (int s = 0; s < M; ++s) {
    need(off + s, b.total_samples);  // mask
    if (feasible_of(key, s)) {
      s0 = s;
      break;
    }
  }
  if (s0 == INT32_MAX) {
    o.status = kBwdEmpty;
    return o;
  }
  // trace check
  for (int k = 0; k < 2 * T; ++k) {
    const int t = trace[k];
    if (t < 0 || t >= M) {
      o.status = kBwdBadTrace;
      return o;
    }
    need(off + t, b.total_samples);
    if (!feasible_of(key, t)) {
      o.status = kBwdBadTrace;
      return o;
    }
  }
  // signature reads every winner's rotation
  for (int i = 0; i <= T; ++i) {
    const int id = i == 0 ? s0 : trace[2 * (i - 1)];
    need(12 * (off + id) + 8, poses_words);
  }
  // active set: the sorted distinct ids of the trace and s0
  std::vector<int> act(kMaxActive);
  int n_act = 0;
  {
    std::vector<int> all(trace.begin(), trace.end());
    all.push_back(s0);
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    if ((int)all.size() > kMaxActive) {
      o.status = kBwdOverflow;
      return o;
    }
    for (int x : all) act[n_act++] = x;
  }
  // rotation checkpoints read by the recomputation
  for (int i = 1; i <= T; ++i) need(ckpt_index(j, (i - 1) / ck, T, ck), (int64_t)b.n * ckpt_count(T, ck));
  need(ckpt_index(j, (T - avg) / ck, T, ck), (int64_t)b.n * ckpt_count(T, ck));
  // radius argmax in the kernel's order: thread tid takes s = r0 + u * 256 +
  // tid, then a butterfly within each wave and a merge over waves
  bool fin = true;
  for (int k = 0; k < 9; ++k) fin = fin && std::isfinite(Rstar[k]);
  std::vector<double> best(kBlock, -1.0);
  std::vector<int> id(kBlock, INT32_MAX);
  for (int r0 = 0; r0 < M; r0 += 4 * kBlock)
    for (int u = 0; u < 4; ++u)
      for (int tid = 0; tid < kBlock; ++tid) {
        const int s = r0 + u * kBlock + tid;
        if (s >= M || !feasible_of(key, s)) continue;
        double R[9];
        sample_rot(key, s, R);
        double f = 0;
        for (int k = 0; k < 9; ++k) f += (Rstar[k] - R[k]) * (Rstar[k] - R[k]);
        radius_take(f, s, best[tid], id[tid]);
      }
  for (int w = 0; w < kBlock / 64; ++w)
    for (int o2 = 32; o2 >= 1; o2 >>= 1) {
      std::vector<double> nb(64);
      std::vector<int> ni(64);
      for (int l = 0; l < 64; ++l) {
        double bb = best[64 * w + l];
        int ii = id[64 * w + l];
        radius_merge(best[64 * w + (l ^ o2)], id[64 * w + (l ^ o2)], bb, ii);
        nb[l] = bb;
        ni[l] = ii;
      }
      for (int l = 0; l < 64; ++l) {
        best[64 * w + l] = nb[l];
        id[64 * w + l] = ni[l];
      }
    }
  double bv = best[0];
  int sD = id[0];
  for (int w = 1; w < kBlock / 64; ++w) radius_merge(best[64 * w], id[64 * w], bv, sD);
  const int sd = sD;  // (the translation search has the same structure)
  if (unguarded) {
    // the code before the guards: insert whatever the search returned
    int ids[2] = {sD, sd};
    for (int e = 0; e < 2; ++e) {
      if (find_sorted(act.data(), n_act, ids[e]) >= 0 || n_act >= kMaxActive) continue;
      int k = n_act++;
      while (k > 0 && act[k - 1] > ids[e]) {
        act[k] = act[k - 1];
        --k;
      }
      act[k] = ids[e];
    }
  } else {
    int32_t st = fin ? kBwdOk : kBwdNonFinite;
    if (st == kBwdOk) st = radius_sample_status(sD, M);
    if (st == kBwdOk) st = radius_sample_status(sd, M);
    if (st == kBwdOk) st = active_insert(act.data(), n_act, kMaxActive, sD, M);
    if (st == kBwdOk) st = active_insert(act.data(), n_act, kMaxActive, sd, M);
    if (st != kBwdOk) {
      o.status = st;
      return o;
    }
  }
  // staging of the active poses, the trace slots, and the per-sample work of
  // the tangent kernels
  for (int a = 0; a < n_act; ++a) need(12 * (off + act[a]) + 11, poses_words);
  for (int k = 0; k < 2 * T; ++k) {
    const int sl = find_sorted(act.data(), n_act, trace[k]);
    need(sl, n_act);
  }
  const int max_dirs = 6 * b.max_kp;
  const int dirs = 6 * I.n_kp;
  for (int a = 0; a < n_act; ++a)
    for (int d = 0; d < dirs; d += 7) {
      need(((int64_t)j * kMaxActive + a) * max_dirs + d, (int64_t)b.n * kMaxActive * max_dirs);  // contrib
      need(((int64_t)j * max_dirs + d) * 27 + 26, (int64_t)b.n * max_dirs * 27);                // tangents
      need(I.kp_off + d / 6, b.total_kp);                                                          // keypoint records
    }
  o.n_act = n_act;
  return o;
}

static std::vector<int> random_trace(Rng &r, uint64_t key, int M, int T, int distinct) {
  std::vector<int> pool;
  while ((int)pool.size() < distinct) {
    int s = (int)(r.next() % (unsigned long long)M);
    if (feasible_of(key, s)) pool.push_back(s);
  }
  std::vector<int> tr(2 * T);
  for (int k = 0; k < 2 * T; ++k) tr[k] = pool[r.next() % pool.size()];
  return tr;
}

int main() {
  Rng r{12345};
  const int T = 4096, avg = 10, ck = ckpt_spacing(5);
  // ---- 64 x 2D-3D, N = 48, 2^20 samples each
  {
    HostBatch b = make_batch(std::vector<int>(64, PURSE_KIND_2D3D), std::vector<int>(64, 48),
                             std::vector<int64_t>(64, 1 << 20));
    const int js[3] = {0, 31, 63};
    for (int j : js) {
      const uint64_t key = b.seed[j];
      const int M = 1 << 20;
      std::vector<int> tr = random_trace(r, key, M, T, 40);
      double Rs[9];
      sample_rot(key ^ 77, 3, Rs);
      Outcome o = run_instance(b, j, record_of(b, j), tr, T, avg, ck, Rs, false, nullptr);
      CHECK(o.status == kBwdOk);
      CHECK(o.indices_ok);
      CHECK(o.n_act >= 2 && o.n_act <= kMaxActive);
      // non-finite centre: stopped with an error before any pose index
      double Rn[9];
      for (int k = 0; k < 9; ++k) Rn[k] = std::nan("");
      o = run_instance(b, j, record_of(b, j), tr, T, avg, ck, Rn, false, nullptr);
      CHECK(o.status == kBwdNonFinite);
      CHECK(o.indices_ok);
      // the same without the guards: the sentinel becomes a sample id
      int64_t bad = -1;
      o = run_instance(b, j, record_of(b, j), tr, T, avg, ck, Rn, true, &bad);
      CHECK(!o.indices_ok);
      CHECK(bad >= 12 * b.total_samples);
      if (j == 0)
        std::printf("unguarded non-finite centre: pose word %lld of %lld (%.1f GB past the array)\n",
                    (long long)bad, (long long)(12 * b.total_samples),
                    4.0 * (double)(bad - 12 * b.total_samples) / 1e9);
      // a trace entry outside the instance, or infeasible
      std::vector<int> t2 = tr;
      t2[100] = M;
      CHECK(run_instance(b, j, record_of(b, j), t2, T, avg, ck, Rs, false, nullptr).status == kBwdBadTrace);
      t2[100] = -1;
      CHECK(run_instance(b, j, record_of(b, j), t2, T, avg, ck, Rs, false, nullptr).status == kBwdBadTrace);
      int inf = 0;
      while (feasible_of(key, inf)) ++inf;
      t2[100] = inf;
      CHECK(run_instance(b, j, record_of(b, j), t2, T, avg, ck, Rs, false, nullptr).status == kBwdBadTrace);
      // more distinct winners than the active set holds
      std::vector<int> t3 = random_trace(r, key, M, T, 600);
      o = run_instance(b, j, record_of(b, j), t3, T, avg, ck, Rs, false, nullptr);
      CHECK(o.status == kBwdOverflow);
      CHECK(o.indices_ok);
      // the record of another instance, and records of random bytes
      o = run_instance(b, j, record_of(b, (j + 1) % 64), tr, T, avg, ck, Rs, false, nullptr);
      CHECK(o.status == kBwdStale);
      for (int trial = 0; trial < 200; ++trial) {
        InstRec g;
        unsigned char *p = reinterpret_cast<unsigned char *>(&g);
        for (size_t k = 0; k < sizeof g; ++k) p[k] = (unsigned char)r.next();
        o = run_instance(b, j, g, tr, T, avg, ck, Rs, false, nullptr);
        CHECK(o.status == kBwdStale);
      }
    }
  }
  // ---- 512 instances, alternating kinds, N ~ U{6..48}, M ~ U{1024..16384}
  {
    std::vector<int> kinds(512), nkp(512);
    std::vector<int64_t> ms(512);
    for (int j = 0; j < 512; ++j) {
      kinds[j] = j & 1;
      nkp[j] = 6 + (int)(r.next() % 43);
      ms[j] = 1024 + (int64_t)(r.next() % 15361);
    }
    HostBatch b = make_batch(kinds, nkp, ms);
    int n_ok = 0;
    for (int j = 0; j < 512; ++j) {
      const uint64_t key = b.seed[j];
      const int M = (int)ms[j];
      std::vector<int> tr = random_trace(r, key, M, T, 3 + (int)(r.next() % 20));
      double Rs[9];
      sample_rot(key ^ 5, 1, Rs);
      Outcome o = run_instance(b, j, record_of(b, j), tr, T, avg, ck, Rs, false, nullptr);
      CHECK(o.status == kBwdOk && o.indices_ok);
      n_ok += o.status == kBwdOk;
      // a record left by a batch with a different layout: instance j's
      // ranges shifted by one keypoint
      InstRec I = record_of(b, j);
      I.kp_off += 1;
      CHECK(run_instance(b, j, I, tr, T, avg, ck, Rs, false, nullptr).status == kBwdStale);
      I = record_of(b, j);
      I.n_samples += 1;
      CHECK(run_instance(b, j, I, tr, T, avg, ck, Rs, false, nullptr).status == kBwdStale);
    }
    std::printf("512-instance batch: %d of 512 instances pass with every index in range\n", n_ok);
  }
  // ---- the batch's own ranges
  {
    HostBatch b = make_batch({0, 1}, {8, 12}, {100, 200});
    InstView v = b.view(1);
    CHECK(inst_view_ok(v));
    v.kp_end = v.total_kp + 1;
    CHECK(!inst_view_ok(v));
    v = b.view(1);
    v.s_end = v.s_off - 1;
    CHECK(!inst_view_ok(v));
    v = b.view(0);
    v.n_kp = PURSE_MAX_KP + 1;
    CHECK(!inst_view_ok(v));
  }
  // ---- fingerprints separate single-bit changes of any input word
  {
    const float a[3] = {0.1f, -0.2f, 0.3f}, c[3] = {320.5f, 240.25f, 0.f}, L[4] = {0.01f, 0.002f, 0.002f, 0.02f};
    uint32_t w[11];
    kp_words(PURSE_KIND_2D3D, a, c, L, 1.f, w);
    const unsigned long long h0 = kp_data_term(3, w);
    for (int k = 0; k < 11; ++k)
      for (int bit = 0; bit < 32; ++bit) {
        uint32_t w2[11];
        std::memcpy(w2, w, sizeof w);
        w2[k] ^= 1u << bit;
        CHECK(kp_data_term(3, w2) != h0);
      }
    CHECK(kp_data_term(4, w) != h0);
  }
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("bwd index guards: all checks passed\n");
  return 0;
}
