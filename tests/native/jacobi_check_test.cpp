// Host run of the float64 Jacobi eigen-solver the library's polar
// decomposition uses (purse_device.hpp, the same template the kernels
// instantiate) on the matrices that made the backward's centre non-finite:
// M^T M for M the sum of rotations about one axis has two equal eigenvalues;
// once the sweeps drive an off-diagonal entry of a pair with bitwise-equal
// diagonal entries below sqrt(smallest normal), the rotation's tangent was
// 2 apq / 0 and the eigenvectors NaN.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "../../paper_2403_09990_amd/csrc/purse_device.hpp"

using namespace purse;

static int g_fail = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                           \
    }                                                                     \
  } while (0)

static bool finite9(const double *A) {
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(A[k])) return false;
  return true;
}

// V^T S0 V is diagonal to rounding and V is orthonormal.
static bool eigen_ok(const double S0[9], const double V[9]) {
  double T[9], VtV[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double t = 0, o = 0;
      for (int a = 0; a < 3; ++a) {
        o += V[3 * a + r] * V[3 * a + c];
        for (int b = 0; b < 3; ++b) t += V[3 * a + r] * S0[3 * a + b] * V[3 * b + c];
      }
      T[3 * r + c] = t;
      VtV[3 * r + c] = o;
    }
  const double scale = std::fabs(S0[0]) + std::fabs(S0[4]) + std::fabs(S0[8]);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      if (r != c && std::fabs(T[3 * r + c]) > 1e-12 * scale) return false;
      if (std::fabs(VtV[3 * r + c] - (r == c ? 1.0 : 0.0)) > 1e-12) return false;
    }
  return true;
}

static void rot_axis(const double e[3], double th, double R[9]) {
  const double c = std::cos(th), s = std::sin(th), v = 1 - c;
  R[0] = c + e[0] * e[0] * v;
  R[1] = e[0] * e[1] * v - e[2] * s;
  R[2] = e[0] * e[2] * v + e[1] * s;
  R[3] = e[1] * e[0] * v + e[2] * s;
  R[4] = c + e[1] * e[1] * v;
  R[5] = e[1] * e[2] * v - e[0] * s;
  R[6] = e[2] * e[0] * v - e[1] * s;
  R[7] = e[2] * e[1] * v + e[0] * s;
  R[8] = c + e[2] * e[2] * v;
}

int main() {
  // 1. the degenerate pair directly: equal diagonal entries, an off-diagonal
  // entry whose square underflows
  {
    const double tiny[4] = {1e-163, -3e-170, 5e-200, 1e-300};
    for (double apq : tiny) {
      double S[9] = {100.0, apq, 0.0, apq, 100.0, 0.0, 0.0, 0.0, 99.0};
      const double S0[9] = {S[0], S[1], S[2], S[3], S[4], S[5], S[6], S[7], S[8]};
      // the rotation as it was: tan = 2 apq / (dl + sqrt(dl^2 + 4 apq^2)) = 2 apq / 0
      const double dl = S[4] - S[0], rt = std::sqrt(dl * dl + 4.0 * apq * apq);
      const double tt_old = 2.0 * apq * (1.0 / (dl + rt));
      const double c_old = 1.0 / std::sqrt(tt_old * tt_old + 1.0), s_old = tt_old * c_old;
      CHECK(!std::isfinite(s_old));
      double V[9];
      jacobi3<double>(S, V, 12);
      CHECK(finite9(V) && finite9(S));
      CHECK(eigen_ok(S0, V));
    }
  }
  // 2. M^T M of sums of rotations about one axis (a double eigenvalue), as the
  // centre of the last iterates of a descent alternating between two winners
  {
    unsigned long long z = 88172645463325252ull;
    auto uni = [&]() {
      z ^= z << 13;
      z ^= z >> 7;
      z ^= z << 17;
      return (z >> 11) * (1.0 / 9007199254740992.0);
    };
    int n_bad = 0, n = 0;
    for (int trial = 0; trial < 200000; ++trial) {
      double e[3] = {uni() - 0.5, uni() - 0.5, uni() - 0.5};
      double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      for (double &x : e) x /= en;
      // with some probability an axis along a coordinate direction, which
      // makes equal diagonal entries likely
      if (trial % 3 == 0) e[0] = 1, e[1] = e[2] = 0;
      if (trial % 3 == 1) e[2] = 1, e[0] = e[1] = 0;
      const double th0 = 6.28 * uni(), dth = 1e-4 * uni();
      double M[9] = {0};
      for (int k = 0; k < 10; ++k) {
        double R[9];
        rot_axis(e, th0 + ((k & 1) ? dth : -dth) / (1.0 + k), R);
        for (int q = 0; q < 9; ++q) M[q] += R[q];
      }
      double S[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) S[3 * r + c] = M[r] * M[c] + M[3 + r] * M[3 + c] + M[6 + r] * M[6 + c];
      const double S0[9] = {S[0], S[1], S[2], S[3], S[4], S[5], S[6], S[7], S[8]};
      double V[9];
      jacobi3<double>(S, V, 12);
      ++n;
      if (!finite9(V) || !eigen_ok(S0, V)) ++n_bad;
    }
    std::printf("sums of rotations about one axis: %d of %d decompositions not finite or not diagonal\n", n_bad, n);
    CHECK(n_bad == 0);
  }
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("jacobi: all checks passed\n");
  return 0;
}
